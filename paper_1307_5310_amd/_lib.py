"""ctypes binding of libstdg.so: argument marshalling only.

Every computation happens in the library's HIP kernels.  Loading fails loudly
when the built library is missing; there is no fallback path.  torch is
imported first so that the library binds to the same HIP runtime as torch's
device memory and streams.
"""
import ctypes
import os

import numpy as np

try:  # torch provides device memory and streams; import it before the library
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - torch is part of the image
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstdg.so")

STDG_OK = 0
STDG_E_NOT_READY = -6
STATUS_NAMES = {0: "STDG_OK", -1: "STDG_E_ARG", -2: "STDG_E_UNSUPPORTED", -3: "STDG_E_NOMEM",
                -4: "STDG_E_DEVICE", -5: "STDG_E_NOT_CONVERGED", -6: "STDG_E_NOT_READY",
                -7: "STDG_E_CAPACITY", -8: "STDG_E_CANCELLED"}
STDG_FP64, STDG_FP32 = 0, 1
STDG_OPERATOR, STDG_RESIDUAL, STDG_OPERATOR_PRECOND = 0, 1, 2


class StdgError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("vertices", ctypes.c_void_p),
                ("n_elements", ctypes.c_int64), ("hexes", ctypes.c_void_p),
                ("p", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("eps", ctypes.c_void_p), ("mu", ctypes.c_void_p),
                ("nsub", ctypes.c_void_p)]


class MeshInfo(ctypes.Structure):
    _fields_ = [("n_elements", ctypes.c_int64), ("n_vertices", ctypes.c_int64),
                ("n_interior_faces", ctypes.c_int64), ("n_boundary_faces", ctypes.c_int64),
                ("trial_size", ctypes.c_int64), ("unknown_size", ctypes.c_int64),
                ("state_size", ctypes.c_int64), ("n_groups", ctypes.c_int32),
                ("n_affine", ctypes.c_int32), ("n_nonaffine", ctypes.c_int32),
                ("n_diagonal_mass", ctypes.c_int32), ("p_max", ctypes.c_int32),
                ("q_max", ctypes.c_int32), ("device_bytes", ctypes.c_int64),
                ("work_order", ctypes.c_int32)]


class Source(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("amp", ctypes.c_double),
                ("center", ctypes.c_double * 3), ("sigma_x", ctypes.c_double),
                ("f0", ctypes.c_double), ("t0", ctypes.c_double), ("sigma_t", ctypes.c_double),
                ("dir", ctypes.c_double * 3)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("inner_prec", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("max_iters", ctypes.c_int32), ("max_refine", ctypes.c_int32),
                ("rtol", ctypes.c_double), ("inner_rtol", ctypes.c_double),
                ("krylov_prec", ctypes.c_int32), ("eta_tol", ctypes.c_double),
                ("eta_t_final", ctypes.c_double), ("use_graph", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("refinements", ctypes.c_int32),
                ("rel_res", ctypes.c_double), ("energy_start", ctypes.c_double),
                ("energy_end", ctypes.c_double), ("eta2", ctypes.c_double)]


class ServeOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_active", ctypes.c_int32),
                ("inner_prec", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("max_iters", ctypes.c_int32), ("max_refine", ctypes.c_int32),
                ("rtol", ctypes.c_double), ("inner_rtol", ctypes.c_double),
                ("krylov_prec", ctypes.c_int32), ("eta_rel", ctypes.c_double),
                ("use_graph", ctypes.c_int32), ("batch_cycles", ctypes.c_int32)]


class GroupInfo(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("q", ctypes.c_int32), ("affine", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("n_elements", ctypes.c_int64)]


class Request(ctypes.Structure):
    _fields_ = [("mesh", MeshDesc), ("t0", ctypes.c_double), ("dt", ctypes.c_double),
                ("n_slabs", ctypes.c_int32), ("source", Source), ("n_modes", ctypes.c_int32),
                ("mnl", ctypes.c_void_p), ("abc", ctypes.c_void_p), ("init_state", ctypes.c_void_p),
                ("c_diss", ctypes.c_double), ("init_state_size", ctypes.c_int64)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("slabs_done", ctypes.c_int32), ("iters", ctypes.c_int64),
                ("max_rel_res", ctypes.c_double), ("energy_start", ctypes.c_double),
                ("energy_end", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("state_size", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("eta_it", ctypes.c_double),
                ("state", ctypes.c_void_p), ("state_capacity", ctypes.c_int64),
                ("batched_cycles", ctypes.c_int64)]


# in the order of the STDG_STRUCT_* indices of stdg_struct_size
STRUCTS = (MeshDesc, MeshInfo, Source, SolveOpts, SolveInfo, ServeOpts, Request, Result, GroupInfo)

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libstdg.so is not built (run __graft_entry__.build()); "
                              "there is no fallback implementation")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "stdg_version": ([], ctypes.c_int),
            "stdg_struct_size": ([i32], ctypes.c_size_t),
            "stdg_last_error": ([], ctypes.c_char_p),
            "stdg_init": ([ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(vp)], ctypes.c_int),
            "stdg_finalize": ([vp], ctypes.c_int),
            "stdg_mesh_upload": ([vp, ctypes.POINTER(MeshDesc), ctypes.POINTER(vp)], ctypes.c_int),
            "stdg_mesh_info": ([vp, ctypes.POINTER(MeshInfo)], ctypes.c_int),
            "stdg_mesh_offsets": ([vp, vp, vp, vp], ctypes.c_int),
            "stdg_mesh_free": ([vp], ctypes.c_int),
            "stdg_mesh_set_dissipation": ([vp, dbl], ctypes.c_int),
            "stdg_mesh_set_order": ([vp, i32], ctypes.c_int),
            "stdg_mesh_set_launch": ([vp, i32, i32], ctypes.c_int),
            "stdg_mesh_group": ([vp, i32, ctypes.POINTER(GroupInfo)], ctypes.c_int),
            "stdg_mesh_autotune": ([vp, ctypes.c_int, dbl, i32, ctypes.POINTER(i32), vp], ctypes.c_int),
            "stdg_residual_apply": ([vp, dbl, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp], ctypes.c_int),
            "stdg_residual_apply_noalloc": ([vp, dbl, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp], ctypes.c_int),
            "stdg_noalloc_scratch_bytes": ([], ctypes.c_size_t),
            "stdg_stream_copy": ([vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
            "stdg_load_assemble": ([vp, ctypes.POINTER(Source), dbl, dbl, vp, vp], ctypes.c_int),
            "stdg_project_modes": ([vp, i32, vp, vp, vp, vp], ctypes.c_int),
            "stdg_slab_solve": ([vp, dbl, dbl, vp, ctypes.POINTER(SolveOpts), vp, vp,
                                 ctypes.POINTER(SolveInfo), vp], ctypes.c_int),
            "stdg_energy": ([vp, vp, ctypes.POINTER(dbl), vp], ctypes.c_int),
            "stdg_residual_dual_norm": ([vp, dbl, vp, ctypes.POINTER(dbl), vp], ctypes.c_int),
            "stdg_serve_start": ([vp, ctypes.POINTER(ServeOpts), ctypes.POINTER(vp)], ctypes.c_int),
            "stdg_serve_submit": ([vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
            "stdg_serve_poll": ([vp, ctypes.c_uint64, ctypes.POINTER(Result)], ctypes.c_int),
            "stdg_serve_clock": ([vp], dbl),
            "stdg_serve_stop": ([vp], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        # the structs mirrored here must match the library's layout
        for which, st in enumerate(STRUCTS):
            if L.stdg_struct_size(which) != ctypes.sizeof(st):
                raise ImportError("libstdg.so struct %s is %d bytes, the binding's %d: rebuild the library"
                                  % (st.__name__, L.stdg_struct_size(which), ctypes.sizeof(st)))
        _lib = L
    return _lib


def exported_symbols():
    """Names declared in include/stdg.h (parsed) that the library must export."""
    import re
    hdr = os.path.join(HERE, "..", "include", "stdg.h")
    text = open(hdr).read()
    return sorted(set(re.findall(r"\b(stdg_[a-z_0-9]+)\s*\(", text)))


def check(status):
    if status != STDG_OK:
        msg = lib().stdg_last_error()
        raise StdgError(status, msg.decode() if msg else "")
    return status


def ptr(x):
    """Device or host address of a torch tensor / numpy array / int / None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


def stream_handle(stream):
    if stream is None:
        if torch is not None and torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream
