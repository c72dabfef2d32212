"""ctypes loader for libfacetransfer.so (argument marshalling only).

The library is built in-tree by ``python -m paper_2504_15814_amd.build``.  A
missing library is an error: there is no fallback implementation.
"""

import ctypes
import os

from .build import lib_path

_LIB = None

c_int64_p = ctypes.POINTER(ctypes.c_int64)
c_double_p = ctypes.POINTER(ctypes.c_double)
c_void_p = ctypes.c_void_p


class PlanBatch(ctypes.Structure):
    """ft_plan_batch"""

    _fields_ = [
        ("op", ctypes.c_void_p),
        ("n_faces", ctypes.c_int64),
        ("orientation", ctypes.c_void_p),
        ("subface", ctypes.c_void_p),
        ("coarse_offset", ctypes.c_void_p),
        ("fine_offset", ctypes.c_void_p),
    ]


# name -> (restype, argtypes); mirrors include/facetransfer.h
SIGNATURES = {
    "build_transfer_operator": (
        ctypes.c_int,
        [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(c_void_p)],
    ),
    "destroy_transfer_operator": (ctypes.c_int, [c_void_p]),
    "interpolate_faces": (
        ctypes.c_int,
        [c_void_p, ctypes.c_int64, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_int, ctypes.c_int,
         c_void_p, ctypes.c_int64, c_void_p, ctypes.c_int64, c_void_p],
    ),
    "restrict_faces": (
        ctypes.c_int,
        [c_void_p, ctypes.c_int64, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_int, ctypes.c_int,
         c_void_p, ctypes.c_int64, c_void_p, ctypes.c_int64, c_void_p],
    ),
    "interpolate_patches": (
        ctypes.c_int,
        [c_void_p, ctypes.c_int64, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_int, ctypes.c_int,
         c_void_p, ctypes.c_int64, c_void_p, ctypes.c_int64, c_void_p],
    ),
    "restrict_patches": (
        ctypes.c_int,
        [c_void_p, ctypes.c_int64, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_int, ctypes.c_int,
         c_void_p, ctypes.c_int64, c_void_p, ctypes.c_int64, c_void_p],
    ),
    "gather_patch_faces": (
        ctypes.c_int,
        [ctypes.c_int, ctypes.c_int, ctypes.c_int64, c_void_p, c_void_p, c_void_p, ctypes.c_int, ctypes.c_int,
         ctypes.c_int, c_void_p, ctypes.c_int64, c_void_p, ctypes.c_int64, c_void_p, c_void_p],
    ),
    "scatter_patch_faces": (
        ctypes.c_int,
        [ctypes.c_int, ctypes.c_int, ctypes.c_int64, c_void_p, c_void_p, c_void_p, ctypes.c_int, ctypes.c_int,
         ctypes.c_int, c_void_p, ctypes.c_int64, c_void_p, ctypes.c_int64, c_void_p, c_void_p],
    ),
    "copy_patch_halos": (
        ctypes.c_int,
        [ctypes.c_int, ctypes.c_int, ctypes.c_int64, c_void_p, c_void_p, c_void_p, ctypes.c_int, ctypes.c_int,
         c_void_p, ctypes.c_int64, c_void_p, c_void_p],
    ),
    "transfer_operator_info": (ctypes.c_int, [c_void_p, c_int64_p, ctypes.c_int]),
    "transfer_operator_segment": (
        ctypes.c_int,
        [c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int64, c_int64_p, c_int64_p, c_double_p, c_int64_p],
    ),
    "transfer_operator_errors": (ctypes.c_int, [c_void_p, c_int64_p, ctypes.c_int]),
    "build_transfer_plan": (
        ctypes.c_int,
        [ctypes.POINTER(PlanBatch), ctypes.c_int, ctypes.c_int, ctypes.c_int, c_void_p, ctypes.c_int64,
         c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(c_void_p)],
    ),
    "run_transfer_plan": (ctypes.c_int, [c_void_p, c_void_p]),
    "run_transfer_batches": (
        ctypes.c_int,
        [ctypes.POINTER(PlanBatch), ctypes.c_int, ctypes.c_int, ctypes.c_int, c_void_p, ctypes.c_int64,
         c_void_p, ctypes.c_int64, ctypes.c_int, c_void_p],
    ),
    "transfer_plan_set_schedule": (ctypes.c_int, [c_void_p, ctypes.c_int64]),
    "transfer_plan_get_schedule": (ctypes.c_int, [c_void_p, c_int64_p]),
    "transfer_plan_autotune": (
        ctypes.c_int, [c_void_p, c_void_p, ctypes.c_int, c_int64_p, ctypes.POINTER(ctypes.c_double)]),
    "destroy_transfer_plan": (ctypes.c_int, [c_void_p]),
    "transfer_plan_capture": (ctypes.c_int, [c_void_p, ctypes.c_int, ctypes.POINTER(c_void_p)]),
    "transfer_plans_capture": (
        ctypes.c_int, [ctypes.POINTER(c_void_p), ctypes.c_int, ctypes.c_int, ctypes.POINTER(c_void_p)]),
    "transfer_graph_launch": (ctypes.c_int, [c_void_p, c_void_p]),
    "destroy_transfer_graph": (ctypes.c_int, [c_void_p]),
    "transfer_last_error": (ctypes.c_char_p, []),
    "transfer_version": (ctypes.c_int, []),
}


def load(path=None):
    """Load (once) and return the ctypes handle of the library."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = path or lib_path()
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m paper_2504_15814_amd.build` "
            "(there is no CPU fallback)"
        )
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def loaded_path():
    return lib_path() if _LIB is not None else None
