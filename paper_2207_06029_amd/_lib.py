"""ctypes binding of liblbib.so (include/lbib.h).  Argument marshalling only: every step of the
method runs in the library's HIP kernels.  Loading fails loudly when the library is missing."""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "liblbib.so")

LBIB_OK = 0
LBIB_NOALLOC_MAX_NODES = 1048576
STATUS = {0: "LBIB_OK", -1: "LBIB_EINVAL", -2: "LBIB_ENOMEM", -3: "LBIB_EDEVICE",
          -4: "LBIB_EUNSTABLE", -5: "LBIB_EBUSY", -6: "LBIB_ENOENT", -7: "LBIB_EDOMAIN"}


class LbibError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class lbib_lattice_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("tau", ctypes.c_double),
                ("bc", ctypes.c_int32 * 6), ("wall_u", (ctypes.c_double * 3) * 6),
                ("body_force", ctypes.c_double * 3)]


class lbib_body_desc(ctypes.Structure):
    _fields_ = [("rigid", ctypes.c_int32), ("integrator", ctypes.c_int32),
                ("ks0", ctypes.c_double), ("thickness", ctypes.c_double),
                ("kb", ctypes.c_double), ("kv", ctypes.c_double),
                ("mass_ratio", ctypes.c_double), ("gravity", ctypes.c_double * 3),
                ("mls_rw", ctypes.c_double), ("mls_alpha", ctypes.c_double),
                ("probe_len", ctypes.c_double), ("shell_h", ctypes.c_double)]


class lbib_job(ctypes.Structure):
    _fields_ = [("lattice", lbib_lattice_desc), ("body", lbib_body_desc),
                ("xyz", ctypes.POINTER(ctypes.c_double)), ("tri", ctypes.POINTER(ctypes.c_int32)),
                ("nv", ctypes.c_int32), ("nt", ctypes.c_int32),
                ("steps", ctypes.c_int64), ("tag", ctypes.c_int64)]


class lbib_batch_opts(ctypes.Structure):
    _fields_ = [("storage", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("tune_cache", ctypes.c_char_p), ("use_graph", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class lbib_server_opts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_int32),
                ("steps_per_tick", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("dry_run", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("slot_nodes", ctypes.c_int64),
                ("slot_vertices", ctypes.c_int32), ("slot_triangles", ctypes.c_int32)]


class lbib_result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("tag", ctypes.c_int64), ("status", ctypes.c_int32),
                ("nv", ctypes.c_int32), ("steps_done", ctypes.c_int64),
                ("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_finish_ns", ctypes.c_int64), ("F", ctypes.c_double * 3),
                ("M", ctypes.c_double * 3), ("xyz", ctypes.POINTER(ctypes.c_double))]


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)

# name -> (restype, argtypes)
SIGNATURES = {
    "lbib_abi_version": (ctypes.c_uint32, []),
    "lbib_last_error": (ctypes.c_char_p, []),
    "lbib_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(lbib_lattice_desc), ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "lbib_lattice_create": (ctypes.c_int, [ctypes.POINTER(lbib_lattice_desc), _P, _P, ctypes.c_size_t, ctypes.POINTER(_P)]),
    "lbib_lattice_destroy": (ctypes.c_int, [_P]),
    "lbib_lattice_init": (ctypes.c_int, [_P, _D, _D]),
    "lbib_body_add": (ctypes.c_int, [_P, ctypes.POINTER(lbib_body_desc), _D, ctypes.c_int32, _I32, ctypes.c_int32, _I32]),
    "lbib_body_set_velocity": (ctypes.c_int, [_P, ctypes.c_int32, _D]),
    "lbib_step": (ctypes.c_int, [_P, ctypes.c_int32]),
    "lbib_stream_only": (ctypes.c_int, [_P, ctypes.c_int32]),
    "lbib_sync": (ctypes.c_int, [_P]),
    "lbib_step_count": (ctypes.c_int64, [_P]),
    "lbib_get_macros": (ctypes.c_int, [_P, _D, _D]),
    "lbib_get_macros_noalloc": (ctypes.c_int, [_P, _D, _D]),
    "lbib_get_populations": (ctypes.c_int, [_P, _D]),
    "lbib_set_populations": (ctypes.c_int, [_P, _D]),
    "lbib_body_get_state": (ctypes.c_int, [_P, ctypes.c_int32, _D, _D]),
    "lbib_body_get_forces": (ctypes.c_int, [_P, ctypes.c_int32, _D, _D, _D]),
    "lbib_body_count": (ctypes.c_int, [_P, ctypes.c_int32, _I32, _I32]),
    "lbib_set_timing": (ctypes.c_int, [_P, ctypes.c_int32]),
    "lbib_kernel_time": (ctypes.c_int, [_P, ctypes.c_int32, _D, _I64]),
    "lbib_batch_create": (ctypes.c_int, [ctypes.POINTER(lbib_job), ctypes.c_int32, ctypes.POINTER(lbib_batch_opts), _P, ctypes.POINTER(_P)]),
    "lbib_batch_destroy": (ctypes.c_int, [_P]),
    "lbib_batch_step": (ctypes.c_int, [_P, ctypes.c_int32]),
    "lbib_batch_sync": (ctypes.c_int, [_P]),
    "lbib_batch_lattice": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(_P)]),
    "lbib_batch_launch_shape": (ctypes.c_int, [_P, _I32, _I32]),
    "lbib_server_create": (ctypes.c_int, [ctypes.POINTER(lbib_server_opts), _P, ctypes.POINTER(_P)]),
    "lbib_server_destroy": (ctypes.c_int, [_P]),
    "lbib_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(lbib_job), ctypes.POINTER(ctypes.c_uint64)]),
    "lbib_server_tick": (ctypes.c_int, [_P]),
    "lbib_server_poll": (ctypes.c_int, [_P, ctypes.POINTER(lbib_result), ctypes.c_int32, _I32]),
    "lbib_server_stats": (ctypes.c_int, [_P, _I32, _I32, ctypes.POINTER(ctypes.c_uint64), _D]),
    "lbib_server_info": (ctypes.c_int, [_P, _I32, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]),
}

_lib = None


def load(path: str = SO):
    """Load liblbib.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with paper_2207_06029_amd.build "
                              "(or __graft_entry__.build())")
        # torch (device memory and streams for callers) ships its own HIP runtime: load it first
        # so that the library binds to that same runtime.  Loaded the other way round, torch
        # would find the system runtime already in the process and fail to initialise.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(rc: int):
    if rc != LBIB_OK:
        raise LbibError(rc, load().lbib_last_error().decode())


def dptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def iptr(a: np.ndarray):
    return a.ctypes.data_as(_I32)
