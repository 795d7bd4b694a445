"""ctypes declarations of the C-ABI in ``include/airhdg.h``.

Loading fails loudly when ``libairhdg.so`` has not been built: there is no
fallback path.
"""
import ctypes as C
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libairhdg.so")

AH_OK, AH_ENOCONV, AH_EINVAL, AH_ESINGULAR, AH_EBREAKDOWN, AH_EHIP, AH_ENOMEM, AH_EUNSUPPORTED = (
    0, 1, -1, -2, -3, -4, -5, -6)
STATUS_NAMES = {0: "AH_OK", 1: "AH_ENOCONV", -1: "AH_EINVAL", -2: "AH_ESINGULAR", -3: "AH_EBREAKDOWN",
                -4: "AH_EHIP", -5: "AH_ENOMEM", -6: "AH_EUNSUPPORTED"}


class HdgParams(C.Structure):
    _fields_ = [("p", C.c_int), ("alpha", C.c_double), ("keep_element_data", C.c_int),
                ("no_block_scale", C.c_int)]


class AirParams(C.Structure):
    _fields_ = [("theta", C.c_double), ("max_coarse", C.c_int), ("max_levels", C.c_int),
                ("relax", C.c_int), ("omega", C.c_double), ("stall", C.c_double),
                ("fp32_cycle", C.c_int), ("adjoint", C.c_int), ("lair_distance", C.c_int),
                ("theta_r", C.c_double), ("order_ratio", C.c_double), ("coarsening", C.c_int),
                ("block_air", C.c_int)]


class SetupInfo(C.Structure):
    _fields_ = [("levels", C.c_int), ("n", C.c_int64 * 32), ("nnz", C.c_int64 * 32),
                ("n_fallback", C.c_int64), ("op_complexity", C.c_double), ("t_setup_ms", C.c_double),
                ("block_view_values", C.c_int64), ("level0_no_interp_pass", C.c_int64)]


class SolveParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int), ("maxit", C.c_int),
                ("precision", C.c_int), ("x0_given", C.c_int), ("method", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("relres", C.c_double),
                ("true_relres", C.c_double), ("t_solve_ms", C.c_double)]


vp = C.c_void_p
i64 = C.c_int64
i32 = C.c_int
dbl = C.c_double
P_i64 = C.POINTER(C.c_int64)
P_i32 = C.POINTER(C.c_int)

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p)

# name -> (restype, argtypes)
SIGNATURES = {
    "ah_last_error": (C.c_char_p, []),
    "ah_set_allocator": (i32, [ALLOC_FN, FREE_FN, vp]),
    "ah_pool_trim": (i32, []),
    "ah_mesh_create": (i32, [i32, i64, vp, i64, vp, C.POINTER(vp)]),
    "ah_mesh_destroy": (None, [vp]),
    "ah_mesh_sizes": (i32, [vp, P_i64, P_i64]),
    "ah_mesh_facets": (i32, [vp, vp, vp]),
    "ah_mesh_boundary_facets": (i32, [vp, vp]),
    "ah_mesh_set_bc": (i32, [vp, vp]),
    "ah_sizes": (i32, [i32, i32, P_i32, P_i32, P_i32, P_i32]),
    "ah_quad_rule": (i32, [i32, i32, vp, vp]),
    "ah_quad_points": (i32, [vp, i32, vp, vp, vp]),
    "ah_quad_points_facets": (i32, [vp, i32, vp, vp]),
    "hdg_assemble_q": (i32, [vp, C.POINTER(HdgParams), dbl, vp, vp, vp, vp, vp, C.POINTER(vp)]),
    "hdg_assemble": (i32, [vp, C.POINTER(HdgParams), dbl, vp, vp, vp, vp, C.POINTER(vp)]),
    "ah_system_destroy": (None, [vp]),
    "ah_system_sizes": (i32, [vp, P_i64, P_i32, P_i64]),
    "ah_system_export": (i32, [vp, vp, vp, vp, vp, vp, vp, vp]),
    "hdg_reconstruct": (i32, [vp, vp, vp, vp]),
    "hdg_inflow_from_trace": (i32, [vp, vp, vp, vp, vp]),
    "hdg_update_neumann": (i32, [vp, vp, vp]),
    "ah_air_defaults": (None, [C.POINTER(AirParams)]),
    "air_setup": (i32, [vp, C.POINTER(AirParams), vp, C.POINTER(vp), C.POINTER(SetupInfo)]),
    "ah_hier_destroy": (None, [vp]),
    "ah_hier_level_sizes": (i32, [vp, i32, P_i64, P_i64, P_i64]),
    "ah_hier_level_export": (i32, [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
    "ah_hier_flow_levels": (i32, [vp, vp, P_i64, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "ah_solve_defaults": (None, [C.POINTER(SolveParams)]),
    "air_solve": (i32, [vp, vp, vp, C.POINTER(SolveParams), vp, C.POINTER(SolveInfo)]),
    "air_solve_adjoint": (i32, [vp, vp, vp, C.POINTER(SolveParams), vp, C.POINTER(SolveInfo)]),
    "air_solve_noalloc": (i32, [vp, vp, vp, C.POINTER(SolveParams), vp, C.POINTER(SolveInfo)]),
    "ah_vcycle_apply": (i32, [vp, vp, vp, i32, i32, vp]),
    "hdg_assemble_grad": (i32, [vp, vp, vp, vp, vp, C.POINTER(C.c_double), vp]),
    "ah_source_gauss": (i32, [i32, i64, vp, i32, vp, dbl, vp, vp, vp]),
    "ah_source_gauss_T": (i32, [i32, i64, vp, i32, vp, dbl, vp, vp, vp]),
    "ah_profile_enable": (None, [i32]),
    "ah_profile_reset": (None, []),
    "ah_profile_read": (i32, [C.c_char_p, P_i64, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
}

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libairhdg.so is not built (run __graft_entry__.build() or "
                               "python paper_2010_11130_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def destroy(name, h, _finalizing=sys.is_finalizing):
    """Call the destructor ``name`` on handle ``h`` from a finaliser.  Skipped
    while the interpreter shuts down (module globals may already be cleared;
    process exit returns the device memory)."""
    if _finalizing() or _lib is None:
        return
    getattr(_lib, name)(h)


class AirHdgError(RuntimeError):
    """A library call failed (``status``); the message is the library's
    ``ah_last_error()`` unless ``msg`` is given."""

    def __init__(self, status, where, msg=None):
        if msg is None:
            msg = lib().ah_last_error().decode(errors="replace")
        super().__init__("%s: %s (%s)" % (where, STATUS_NAMES.get(status, status), msg))
        self.status = status


def check(status, where, allow=(AH_OK,)):
    if status not in allow:
        raise AirHdgError(status, where)
    return status
