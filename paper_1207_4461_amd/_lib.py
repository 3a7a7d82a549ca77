"""ctypes binding of libqbx.so (include/qbx.h): argument marshalling only.

The library is the in-tree ``libqbx.so`` built by ``paper_1207_4461_amd.build``
(or the file QBX_LIB names, such as the sanitizer build); loading fails loudly
when it is missing (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("QBX_LIB") or os.path.join(HERE, "libqbx.so")

QBX_TUNE_FORWARD, QBX_TUNE_TAPE, QBX_TUNE_ADJOINT, QBX_TUNE_FUSED, QBX_TUNE_ALL = 1, 2, 4, 8, 15
QBX_TIMER_CLASSES = 9   # entries qbx_kernel_timer_read writes
QBX_OK = 0
QBX_EINVAL = -1
QBX_EWORKSPACE = -2
QBX_EORIENT = -3
QBX_EGRAF = -4
QBX_EDEVICE = -5
QBX_EIO = -6

QBX_S = 1
QBX_D = 2
QBX_INTERIOR = -1
QBX_BOTH = 0
QBX_EXTERIOR = 1
QBX_Q = 16
QBX_PMAX = 24
QBX_OVERSAMPLE_MAX = 8
QBX_STATIC_SCRATCH_BYTES = 64 << 20   # the no-workspace forward's device array

class QBXError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libqbx error {code}: {msg}")
        self.code = code


class Geometry(C.Structure):
    _fields_ = [("n_panels", C.c_int32), ("q", C.c_int32), ("nodes", C.c_void_p)]


class ForwardOptions(C.Structure):
    """qbx_forward_options of include/qbx.h."""
    _fields_ = [("dipole", C.c_int32), ("center_rule", C.c_int32)]


class BatchItem(C.Structure):
    """qbx_batch_item of include/qbx.h."""
    _fields_ = [("node_offset", C.c_int64), ("density_offset", C.c_int64),
                ("out_offset", C.c_int64), ("n_panels", C.c_int32), ("p", C.c_int32),
                ("kind", C.c_int32), ("side", C.c_int32), ("k", C.c_double), ("r", C.c_double)]


class Tuning(C.Structure):
    """qbx_tuning of include/qbx.h."""
    _fields_ = [("forward_waves", C.c_int32), ("tape_waves", C.c_int32),
                ("adjoint_waves", C.c_int32), ("batch_adjoint_tasks", C.c_int32),
                ("batch_grid_scale", C.c_double), ("fused_tiles", C.c_int32),
                ("batch_fused_chunks", C.c_int32), ("fused_part_bytes", C.c_double)]


_lib = None


def load() -> C.CDLL:
    """Load libqbx.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1207_4461_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    vp, dbl, i32, sz = C.c_void_p, C.c_double, C.c_int, C.c_size_t
    gp = C.POINTER(Geometry)
    sig = {
        "qbx_workspace_bytes": (sz, [i32, i32, i32, i32, i32, i32]),
        "qbx_tape_bytes": (sz, [i32, i32, i32, i32, i32]),
        "qbx_layer_potential": (i32, [gp, vp, dbl, i32, dbl, i32, i32, i32, vp, vp, vp, sz, vp]),
        "qbx_layer_potential_noalloc": (i32, [gp, vp, dbl, i32, dbl, i32, i32, i32, vp, vp]),
        "qbx_layer_potential_gradient": (i32, [gp, vp, dbl, i32, dbl, i32, i32, i32, vp, vp, vp,
                                               sz, vp]),
        "qbx_solve_workspace_bytes": (sz, [i32, i32, i32, i32, i32, i32]),
        "qbx_solve_dirichlet": (i32, [gp, vp, dbl, i32, dbl, i32, i32, dbl, dbl, dbl, dbl, i32,
                                      i32, vp, C.POINTER(i32), C.POINTER(dbl), vp, sz, vp]),
        "qbx_layer_potential_ext": (i32, [gp, vp, dbl, i32, dbl, i32, i32, i32,
                                          C.POINTER(ForwardOptions), vp, vp, sz, vp]),
        "qbx_solve_dirichlet_adjoint": (i32, [gp, vp, dbl, i32, dbl, i32, i32, dbl, dbl, dbl,
                                              dbl, i32, i32, vp, C.POINTER(i32),
                                              C.POINTER(dbl), vp, sz, vp]),
        "qbx_layer_potential_split_gradient": (i32, [gp, vp, dbl, i32, dbl, i32, i32, i32, dbl,
                                                     vp, vp, vp, sz, vp]),
        "qbx_layer_potential_split_adjoint": (i32, [gp, vp, dbl, i32, dbl, i32, i32, i32, dbl,
                                                    vp, vp, vp, vp, sz, vp]),
        "qbx_layer_potential_split": (i32, [gp, vp, dbl, i32, dbl, i32, i32, i32, dbl, vp, vp,
                                            sz, vp]),
        "qbx_layer_potential_adjoint": (i32, [gp, vp, dbl, i32, dbl, i32, i32, i32, vp, vp, vp,
                                              vp, vp, sz, vp]),
        "qbx_check_geometry": (i32, [gp, i32, dbl, i32, i32, C.POINTER(dbl), C.POINTER(dbl), vp,
                                     sz, vp]),
        "qbx_signed_area_host": (i32, [vp, i32, C.POINTER(dbl)]),
        "qbx_strerror": (C.c_char_p, [i32]),
        "qbx_last_error": (C.c_char_p, []),
        "qbx_debug_hankel01": (i32, [vp, i32, vp, vp, vp]),
        "qbx_debug_besselj": (i32, [vp, i32, i32, vp, vp]),
        "qbx_kernel_timer": (i32, [i32]),
        "qbx_principal_value": (i32, [vp, vp, i32, i32, i32, vp, vp]),
        "qbx_gradient_principal_value": (i32, [gp, vp, i32, i32, vp, vp, vp, vp, vp]),
        "qbx_batched_workspace_bytes": (sz, [C.POINTER(BatchItem), i32, i32]),
        "qbx_batched_tape_bytes": (sz, [C.POINTER(BatchItem), i32]),
        "qbx_layer_potential_batched": (i32, [C.POINTER(BatchItem), i32, vp, vp, vp, vp, i32, vp,
                                              sz, vp]),
        "qbx_layer_potential_batched_adjoint": (i32, [C.POINTER(BatchItem), i32, vp, vp, vp, vp,
                                                      vp, vp, i32, vp, sz, vp]),
        "qbx_kernel_timer_read": (i32, [C.POINTER(dbl), C.POINTER(i32)]),
        "qbx_explicit_workspace_bytes": (sz, [i32, i32, i32, i32]),
        "qbx_explicit_tape_bytes": (sz, [i32, i32]),
        "qbx_apply_explicit": (i32, [i32, vp, vp, vp, i32, vp, vp, vp, dbl, i32, i32, vp, vp, vp,
                                     sz, vp]),
        "qbx_expansion_workspace_bytes": (sz, [i32, i32, i32, i32, i32, i32]),
        "qbx_expansion_coefficients": (i32, [gp, vp, dbl, i32, dbl, i32, i32, i32, vp, vp, vp, vp,
                                             sz, vp]),
        "qbx_evaluate_expansions": (i32, [i32, vp, vp, dbl, i32, i32, i32, vp, vp, vp, vp]),
        "qbx_assign_centers": (i32, [i32, vp, vp, i32, vp, dbl, vp, vp]),
        "qbx_apply_explicit_gradient": (i32, [i32, vp, vp, vp, i32, vp, vp, vp, dbl, i32, i32,
                                              vp, vp, sz, vp]),
        "qbx_apply_explicit_adjoint": (i32, [i32, vp, vp, vp, i32, vp, vp, vp, dbl, i32, i32, vp,
                                             vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]),
        "qbx_set_tuning": (i32, [C.POINTER(Tuning)]),
        "qbx_get_tuning": (i32, [C.POINTER(Tuning)]),
        "qbx_solve_node_gradient_workspace_bytes": (sz, [i32, i32, i32, i32]),
        "qbx_solve_dirichlet_node_gradient": (i32, [gp, vp, vp, dbl, i32, dbl, i32, i32, dbl, dbl,
                                                    dbl, vp, vp, sz, vp]),
        "qbx_autotune_workspace_bytes": (sz, [i32, i32, i32, i32, i32, i32]),
        "qbx_autotune": (i32, [gp, vp, dbl, i32, dbl, i32, i32, i32, i32, i32, C.c_char_p,
                               C.POINTER(Tuning), vp, sz, vp]),
        "qbx_autotune_batched_workspace_bytes": (sz, [C.POINTER(BatchItem), i32, i32]),
        "qbx_autotune_batched": (i32, [C.POINTER(BatchItem), i32, vp, vp, i32, i32, i32,
                                       C.c_char_p, C.POINTER(Tuning), vp, sz, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != QBX_OK:
        lib = load()
        raise QBXError(rc, f"{lib.qbx_strerror(rc).decode()}: {lib.qbx_last_error().decode()}")
