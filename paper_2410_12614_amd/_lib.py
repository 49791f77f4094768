"""ctypes declarations of the C ABI in ``include/fe.h``.

Loading fails loudly (``FeLibraryError``) when ``libfe.so`` has not been
built: there is no fallback implementation of any step.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfe.so")

# status codes
FE_OK = 0
FE_EINVAL = -1
FE_EUNSUPPORTED = -2
FE_EOVERFLOW = -3
FE_EHIP = -4
FE_EDEGENERATE = -5
FE_ESIZE = -6

FE_TRIANGLE = 2
FE_TETRAHEDRON = 3
FE_HEXAHEDRON = 8
FE_MASS = 0
FE_STIFFNESS = 1
FE_FP64 = 0
FE_FP32 = 1
FE_FP16_ACC32 = 2
FE_BF16_ACC32 = 3
FE_SPLITFP16_ACC32 = 4
FE_GEOM_FP64 = 0
FE_GEOM_FP32 = 1
FE_GEOM_AUTO = 2
FE_SYMBOLIC_COUNT = 0
FE_SYMBOLIC_FILL = 1
FE_NUMERIC = 2
FE_NUMERIC_GATHER = 3
FE_NUMERIC_GEOMETRY = 4
FE_NUMERIC_FUSED = 5
FE_NUMERIC_LOCAL = 6
FE_NUMERIC_ASSEMBLE = 7
FE_ACTION = 0
FE_VJP = 1

# every symbol declared in include/fe.h
EXPORTS = (
    "fe_tabulate",
    "fe_form_prepare",
    "fe_cell_kernels",
    "fe_cell_kernels_tile",
    "fe_tune_cell_kernels",
    "fe_dg_pattern",
    "fe_assemble_csr",
    "fe_assemble_csr_noalloc",
    "fe_vector_plan",
    "fe_action_vjp",
    "fe_get_device_status",
    "fe_status_string",
    "fe_version",
)


class FeLibraryError(RuntimeError):
    pass


class fe_form_desc(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("cell", "degree", "quad_degree", "form", "has_coeff", "precision", "geom_precision")]


class fe_mesh_view(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int64), ("cell_coords", ctypes.c_void_p),
                ("dofmap", ctypes.c_void_p), ("n_dofs", ctypes.c_int64),
                ("coeff", ctypes.c_void_p)]


class fe_csr(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("nnz", ctypes.c_int64), ("max_row_len", ctypes.c_int64),
                ("schedule", ctypes.c_int64), ("schedule_span", ctypes.c_int32),
                ("schedule_elt", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("values", ctypes.c_void_p)]


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FeLibraryError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2410_12614_amd.build` "
            "(there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32 = ctypes.c_int32
    lib.fe_tabulate.argtypes = [i32, i32, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), P, P, P]
    lib.fe_tabulate.restype = i32
    lib.fe_form_prepare.argtypes = [ctypes.POINTER(fe_form_desc), P, ctypes.POINTER(ctypes.c_size_t), P]
    lib.fe_form_prepare.restype = i32
    lib.fe_cell_kernels.argtypes = [ctypes.POINTER(fe_form_desc), P, ctypes.POINTER(fe_mesh_view), P, P]
    lib.fe_cell_kernels.restype = i32
    lib.fe_cell_kernels_tile.argtypes = [ctypes.POINTER(fe_form_desc), P,
                                         ctypes.POINTER(fe_mesh_view), P, i32, P]
    lib.fe_cell_kernels_tile.restype = i32
    lib.fe_tune_cell_kernels.argtypes = [ctypes.POINTER(fe_form_desc), P,
                                         ctypes.POINTER(fe_mesh_view), P, i32,
                                         ctypes.POINTER(i32), P, P]
    lib.fe_tune_cell_kernels.restype = i32
    lib.fe_dg_pattern.argtypes = [i32, P, P, P, P, ctypes.POINTER(ctypes.c_int64), P]
    lib.fe_dg_pattern.restype = i32
    lib.fe_assemble_csr.argtypes = [ctypes.POINTER(fe_form_desc), ctypes.POINTER(P), i32,
                                    ctypes.POINTER(fe_mesh_view), i32, ctypes.POINTER(fe_csr), P,
                                    ctypes.POINTER(ctypes.c_size_t), P,
                                    ctypes.POINTER(ctypes.c_size_t), P]
    lib.fe_assemble_csr.restype = i32
    lib.fe_assemble_csr_noalloc.argtypes = [ctypes.POINTER(fe_form_desc), ctypes.POINTER(P), i32,
                                            ctypes.POINTER(fe_mesh_view), ctypes.POINTER(fe_csr), P, P]
    lib.fe_assemble_csr_noalloc.restype = i32
    lib.fe_vector_plan.argtypes = [ctypes.POINTER(fe_mesh_view), i32, P,
                                   ctypes.POINTER(ctypes.c_size_t), P]
    lib.fe_vector_plan.restype = i32
    lib.fe_action_vjp.argtypes = [ctypes.POINTER(fe_form_desc), P, ctypes.POINTER(fe_mesh_view), P,
                                  i32, P, P, P, P, P, P, ctypes.POINTER(ctypes.c_size_t), P]
    lib.fe_action_vjp.restype = i32
    lib.fe_get_device_status.argtypes = [P, P]
    lib.fe_get_device_status.restype = i32
    lib.fe_status_string.argtypes = [i32]
    lib.fe_status_string.restype = ctypes.c_char_p
    lib.fe_version.argtypes = []
    lib.fe_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


class FeError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = load().fe_status_string(status).decode()
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


def check(status: int, where: str) -> None:
    if status != FE_OK:
        raise FeError(status, where)
