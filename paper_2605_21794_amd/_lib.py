"""ctypes declarations of the C ABI in include/vp.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, c_char_p, c_double, c_int32, c_int64, c_size_t,
                    c_void_p)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvp.so")

VP_OK, VP_ERR_ARG, VP_ERR_HIP, VP_ERR_NONFINITE, VP_ERR_STATE, VP_ERR_RANGE = range(6)
VP_FP64, VP_FP32_COMP, VP_FP32, VP_FP32_TWOSUM = 0, 1, 2, 3
VP_ABI_VERSION = 10         # the layout of the structures declared below
VP_SLOT_OCCUPIED, VP_SLOT_NONFINITE = 1, 2
VP_SOLVE_SCAN, VP_SOLVE_FFT = 0, 1
VP_PROJ_ELEM, VP_PROJ_NODAL, VP_PROJ_CONSISTENT = 0, 1, 2
VP_MIN_NG, VP_MAX_NG = 8, 1024
VP_MAX_SORT_CHUNK_F32, VP_MAX_SORT_CHUNK_F64 = 4096, 2048
VP_MAX_ACC_COPIES = 8


class vp_config(Structure):
    _fields_ = [("n", c_int64), ("ng", c_int32), ("precision", c_int32), ("L", c_double),
                ("dt", c_double), ("sort_every", c_int32), ("sort_chunk", c_int32),
                ("hist_cap", c_int32), ("solver", c_int32),
                ("projection", c_int32), ("monopole_only", c_int32),
                ("no_self_field", c_int32), ("ext_mode", c_int32), ("ext_amplitude", c_double),
                ("element_order", c_int32), ("moment_order", c_int32)]


class vp_particles(Structure):
    _fields_ = [("Q", c_void_p), ("P", c_void_p), ("qs", c_void_p), ("ps", c_void_p),
                ("psi", c_void_p), ("Mqq", c_void_p), ("Mqp", c_void_p), ("Mpp", c_void_p)]


class vp_diag(Structure):
    _fields_ = [("step", c_int64), ("t", c_double), ("K", c_double), ("W", c_double),
                ("H", c_double), ("charge", c_double), ("momentum", c_double),
                ("e_amp", c_double), ("e1_re", c_double), ("e1_im", c_double), ("U", c_double),
                ("stamp", c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class vp_tuning(Structure):
    _fields_ = [("threads", c_int32), ("ppt", c_int32), ("acc_copies", c_int32),
                ("use_graph", c_int32), ("graph_steps", c_int32), ("persistent", c_int32),
                ("wave_reduce", c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


H = c_void_p  # vp_handle*

# name -> (restype, argtypes); every symbol declared in include/vp.h
SIGNATURES = {
    "vp_workspace_bytes": (c_int32, [POINTER(vp_config), POINTER(c_size_t)]),
    "vp_create": (c_int32, [POINTER(vp_config), vp_particles, c_void_p, c_void_p, POINTER(H)]),
    "vp_engine_create": (c_int32, [c_int32, c_int32, c_void_p, POINTER(H)]),
    "vp_create_batch": (c_int32, [c_int32, POINTER(vp_config), POINTER(vp_particles),
                                  POINTER(c_void_p), c_void_p, POINTER(H)]),
    "vp_admit": (c_int32, [H, c_int32, POINTER(vp_config), vp_particles, c_void_p]),
    "vp_retire": (c_int32, [H, c_int32]),
    "vp_destroy": (c_int32, [H]),
    "vp_deposit": (c_int32, [H]),
    "vp_poisson": (c_int32, [H]),
    "vp_gather_push": (c_int32, [H, c_double, c_double]),
    "vp_step": (c_int32, [H, c_int32]),
    "vp_sync_state": (c_int32, [H]),
    "vp_sort": (c_int32, [H, c_int32, c_void_p]),
    "vp_cell_index": (c_int32, [H, c_int32, c_void_p]),
    "vp_diagnostics": (c_int32, [H, c_int32, POINTER(vp_diag), c_void_p]),
    "vp_history": (c_int32, [H, c_int32, c_int64, c_int32, POINTER(vp_diag)]),
    "vp_set_tuning": (c_int32, [H, POINTER(vp_tuning)]),
    "vp_get_tuning": (c_int32, [H, POINTER(vp_tuning)]),
    "vp_tune_scratch_bytes": (c_int32, [H, POINTER(c_size_t)]),
    "vp_tune": (c_int32, [H, c_void_p, c_int32, POINTER(vp_tuning), POINTER(c_double)]),
    "vp_occupancy": (c_int32, [H, POINTER(c_int32), POINTER(c_int64)]),
    "vp_slot_status": (c_int32, [H, c_int32, POINTER(c_int64), POINTER(c_int32)]),
    "vp_cluster_workspace_bytes": (c_int32, [c_int64, c_int32, POINTER(c_size_t)]),
    "vp_cluster_markers": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_int32, c_void_p,
                                     c_int32, c_double, c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_void_p, c_void_p, c_void_p,
                                     POINTER(c_int32)]),
    "vp_cluster_minibatch_workspace_bytes": (c_int32, [c_int64, c_int32, c_int32,
                                                       POINTER(c_size_t)]),
    "vp_cluster_markers_static": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_int32,
                                            c_void_p, c_int32, c_double, c_void_p, c_void_p,
                                            c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                            POINTER(c_int32)]),
    "vp_cluster_markers_minibatch": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_int32,
                                               c_void_p, c_void_p, c_int32, c_int32, c_double,
                                               c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                               c_void_p, c_void_p, c_void_p, c_void_p,
                                               POINTER(c_int32)]),
    "vp_status_string": (c_char_p, [c_int32]),
    "vp_last_error": (c_char_p, []),
    "vp_wall_clock_hz": (c_int32, [POINTER(c_double)]),
    "vp_prepare_step": (c_int32, [H, c_int32]),
    "vp_abi_version": (c_int32, []),
}

_lib = None


class VPError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        self.status = status
        super().__init__(f"{func} -> status {status}: {msg}")


def _hip_runtime_paths():
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    paths.add(line.split()[-1])
    except OSError:
        pass
    return sorted(paths)


def load(path: str = LIB_PATH):
    """Load libvp.so (after torch, so both share the HIP runtime torch already loaded)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is missing: build it with `python -m paper_2605_21794_amd.build`")
    import torch  # noqa: F401  (brings in torch's HIP runtime first)
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.vp_abi_version() != VP_ABI_VERSION:
        raise RuntimeError(f"{path} has ABI version {lib.vp_abi_version()}, these bindings "
                           f"expect {VP_ABI_VERSION}: rebuild it")
    runtimes = _hip_runtime_paths()
    if len(runtimes) > 1:
        raise RuntimeError(f"two HIP runtimes loaded in one process: {runtimes}")
    _lib = lib
    return lib


def check(status: int, func: str):
    if status != VP_OK:
        msg = _lib.vp_last_error().decode() if _lib is not None else ""
        raise VPError(status, func, msg)
