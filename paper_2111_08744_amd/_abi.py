"""ctypes declarations of the C ABI in include/mpath.h (argument marshalling only).

The shared library is loaded from this package's directory; importing this
module raises when it is missing, so nothing can silently fall back to
another implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpath.so")

MPATH_OK = 0
MPATH_ERR_INVALID_ARG = -1
MPATH_ERR_NOT_FULL_TREE = -2
MPATH_ERR_WORKSPACE_TOO_SMALL = -3
MPATH_ERR_DEVICE = -4
MPATH_ERR_UNSUPPORTED = -5

MPATH_RAY_REACHED = 0
MPATH_RAY_LEFT_DOMAIN = 1
MPATH_RAY_MAX_STEPS = 2
MPATH_RAY_NONFINITE = 3

MPATH_F64 = 0
MPATH_F32 = 1
MPATH_STOP_REDSHIFT = 0
MPATH_STOP_CHI = 1
MPATH_SURFACE_ETA, MPATH_SURFACE_CHI, MPATH_SURFACE_LAMBDA, MPATH_SURFACE_Z = 0, 1, 2, 3
MPATH_DPHIDL_CHAIN, MPATH_DPHIDL_DIFF = 0, 1
MPATH_SCHED_AUTO = 0
MPATH_SCHED_STATIC = 1
MPATH_SCHED_PERSISTENT = 2


class mpath_cosmo(C.Structure):
    _fields_ = [("omega_m", C.c_double), ("omega_l", C.c_double), ("h", C.c_double)]


class mpath_grid_desc(C.Structure):
    _fields_ = [("box", C.c_double), ("n0", C.c_int32), ("max_level", C.c_int32),
                ("periodic", C.c_int32), ("value_dtype", C.c_int32), ("n_cells", C.c_int64),
                ("level", C.c_void_p), ("ijk", C.c_void_p), ("phi", C.c_void_p), ("grad", C.c_void_p),
                ("dphi_deta", C.c_void_p)]


class mpath_grid_info(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n0", C.c_int32), ("max_level", C.c_int32),
                ("periodic", C.c_int32), ("box", C.c_double), ("eta0", C.c_double),
                ("cells_per_level", C.c_int64 * 16), ("payload", C.c_void_p), ("perm", C.c_void_p)]


class mpath_cast_desc(C.Structure):
    _fields_ = [("n_obs", C.c_int32), ("obs_pos", C.c_void_p), ("stop_value", C.c_void_p),
                ("stop_kind", C.c_int32), ("nside", C.c_int32), ("pix_first", C.c_void_p),
                ("pix_count", C.c_void_p), ("order", C.c_int32), ("steps_per_cell", C.c_int32),
                ("adaptive", C.c_int32), ("max_steps", C.c_int64), ("schedule", C.c_int32),
                ("block_size", C.c_int32), ("waves_per_cu", C.c_int32), ("batch", C.c_int32),
                ("checkpoint_every", C.c_int32), ("dirs", C.c_void_p), ("n_surfaces", C.c_int32),
                ("surface_stops", C.c_void_p), ("stop_surface", C.c_int32), ("dphidl", C.c_int32)]


class mpath_observables(C.Structure):
    _fields_ = [("beta", C.c_void_p), ("alpha", C.c_void_p), ("z5", C.c_void_p), ("z0", C.c_void_p),
                ("phi_src", C.c_void_p), ("n_steps", C.c_void_p), ("status", C.c_void_p),
                ("hash", C.c_void_p), ("chi", C.c_void_p), ("z1", C.c_void_p), ("z4", C.c_void_p),
                ("isw", C.c_void_p)]


class mpath_adjoint_desc(C.Structure):
    _fields_ = [("dL_dalpha", C.c_void_p), ("dL_dz", C.c_void_p), ("jac", C.c_void_p),
                ("dz_dtheta", C.c_void_p), ("dL_dvalues", C.c_void_p), ("dL_dphi_total", C.c_void_p),
                ("ray_status", C.c_void_p)]


class mpath_finder_desc(C.Structure):
    _fields_ = [("obs_pos", C.c_void_p), ("n_src", C.c_int64), ("src_pos", C.c_void_p), ("order", C.c_int32),
                ("steps_per_cell", C.c_int32), ("adaptive", C.c_int32), ("max_steps", C.c_int64),
                ("tol", C.c_double), ("max_iter", C.c_int32), ("identity_iters", C.c_int32),
                ("checkpoint_every", C.c_int32), ("grid_rounds", C.c_int32),
                ("grid_n", C.c_int32), ("grid_max", C.c_int64)]


class mpath_finder_out(C.Structure):
    _fields_ = [("theta", C.c_void_p), ("A", C.c_void_p), ("dz_dtheta", C.c_void_p), ("z5", C.c_void_p),
                ("z0", C.c_void_p), ("phi_src", C.c_void_p), ("sep", C.c_void_p), ("n_iter", C.c_void_p),
                ("status", C.c_void_p), ("z1", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"the HIP library is not built: {LIB_PATH} "
                              "(run `python -m paper_2111_08744_amd.build`)")
        L = C.CDLL(LIB_PATH)
        P, vp, sz = C.POINTER, C.c_void_p, C.c_size_t
        L.mpath_grid_workspace_bytes.argtypes = [P(mpath_grid_desc), P(sz)]
        L.mpath_grid_build.argtypes = [P(mpath_grid_desc), P(mpath_cosmo), vp, sz, vp, P(vp)]
        L.mpath_grid_aux_bytes.argtypes = [P(mpath_grid_desc), P(sz)]
        L.mpath_grid_build_with_aux.argtypes = [P(mpath_grid_desc), P(mpath_cosmo), vp, sz, vp, sz, vp, P(vp)]
        L.mpath_grid_free.argtypes = [vp]
        L.mpath_grid_get_info.argtypes = [vp, P(mpath_grid_info)]
        L.mpath_grid_set_values.argtypes = [vp, vp, vp]
        L.mpath_cast_workspace_bytes.argtypes = [vp, P(mpath_cast_desc), P(sz)]
        L.mpath_cast.argtypes = [vp, P(mpath_cast_desc), P(mpath_observables), vp, sz, vp]
        L.mpath_cast_count_rays.argtypes = [P(mpath_cast_desc), P(C.c_int64)]
        L.mpath_cast_noalloc.argtypes = [vp, P(mpath_cast_desc), P(mpath_observables), vp]
        L.mpath_cast_jacobian_workspace_bytes.argtypes = [vp, P(mpath_cast_desc), P(sz)]
        L.mpath_cast_jacobian.argtypes = [vp, P(mpath_cast_desc), P(mpath_observables), vp, vp, vp, sz, vp]
        L.mpath_adjoint_workspace_bytes.argtypes = [vp, P(mpath_cast_desc), P(sz)]
        L.mpath_adjoint.argtypes = [vp, P(mpath_cast_desc), P(mpath_observables), vp, sz,
                                    P(mpath_adjoint_desc), vp, sz, vp]
        L.mpath_autotune_workspace_bytes.argtypes = [vp, P(mpath_cast_desc), C.c_int32, P(sz)]
        L.mpath_autotune.argtypes = [vp, P(mpath_cast_desc), C.c_int32, vp, sz, vp, P(mpath_cast_desc),
                                     P(C.c_float)]
        L.mpath_lensing_maps.argtypes = [vp, C.c_int64, vp, vp]
        L.mpath_finite_beam_workspace_bytes.argtypes = [vp, P(mpath_cast_desc), P(sz)]
        L.mpath_finite_beam.argtypes = [vp, P(mpath_cast_desc), C.c_double, vp, vp, vp, sz, vp]
        L.mpath_infinitesimal_beam.argtypes = [vp, P(mpath_cast_desc), P(mpath_observables), vp, vp, sz, vp]
        L.mpath_find_geodesics_workspace_bytes.argtypes = [vp, P(mpath_finder_desc), P(sz)]
        L.mpath_find_geodesics.argtypes = [vp, P(mpath_finder_desc), P(mpath_finder_out), vp, sz, vp]
        L.mpath_born_beam.argtypes = [vp, P(mpath_cast_desc), vp, vp, vp, sz, vp]
        L.mpath_gather_probe.argtypes = [vp, sz, C.c_int32, C.c_int32, C.c_int64, C.c_int32, C.c_uint32, vp, vp]
        L.mpath_double_layer.argtypes = [C.c_int64, vp, vp, vp, vp, P(mpath_cosmo), vp]
        L.mpath_healpix_dirs.argtypes = [C.c_int32, C.c_int64, C.c_int64, vp, vp]
        L.mpath_status_string.restype = C.c_char_p
        L.mpath_status_string.argtypes = [C.c_int]
        L.mpath_last_error.restype = C.c_char_p
        L.mpath_version.restype = C.c_char_p
        for name in ("mpath_grid_workspace_bytes", "mpath_grid_build", "mpath_grid_free",
                     "mpath_grid_aux_bytes", "mpath_grid_build_with_aux",
                     "mpath_grid_get_info", "mpath_grid_set_values", "mpath_cast_workspace_bytes",
                     "mpath_cast", "mpath_cast_count_rays", "mpath_cast_noalloc", "mpath_adjoint_workspace_bytes",
                     "mpath_cast_jacobian_workspace_bytes", "mpath_cast_jacobian",
                     "mpath_adjoint", "mpath_autotune_workspace_bytes", "mpath_autotune", "mpath_gather_probe",
                     "mpath_lensing_maps", "mpath_finite_beam_workspace_bytes", "mpath_finite_beam",
                     "mpath_infinitesimal_beam", "mpath_find_geodesics_workspace_bytes", "mpath_find_geodesics",
                     "mpath_born_beam", "mpath_double_layer", "mpath_healpix_dirs"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


class MpathError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = lib().mpath_last_error().decode(errors="replace")
        super().__init__(f"{where}: {lib().mpath_status_string(code).decode()} ({code}): {msg}")


def check(code, where):
    if code != MPATH_OK:
        raise MpathError(code, where)
