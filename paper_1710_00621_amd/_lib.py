"""ctypes loader for libcrsolve.so (argument marshalling only).

torch is imported first so that the library binds to the HIP runtime torch
already loaded (one HIP/HSA runtime per process).  A missing library is a
hard error: there is no fallback path.
"""
import ctypes
import os

import torch  # noqa: F401  (load torch's HIP runtime before the library)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcrsolve.so")

c_double_p = ctypes.POINTER(ctypes.c_double)
c_int_p = ctypes.POINTER(ctypes.c_int)
c_int64_p = ctypes.POINTER(ctypes.c_int64)
vp = ctypes.c_void_p

CRS_OK = 0
CRS_EINVAL = -1
CRS_ENOMEM = -2
CRS_EHIP = -3
CRS_ENOTCONV = -4
CRS_EBREAKDOWN = -5
CRS_EUNSUPPORTED = -6

PRECOND = {"none": 0, "diag": 1, "pinv": 2, "add": 3}
MODE = {"wf": 0, "cr": 1}


class CrsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"crsolve error {status}: {msg}")
        self.status = status


class BandDesc(ctypes.Structure):
    _fields_ = [("grid", vp), ("lmax", ctypes.c_int), ("beam", c_double_p),
                ("tau", c_double_p), ("q", c_double_p)]


class MaskOpts(ctypes.Structure):
    _fields_ = [("lowpass_r2", ctypes.c_double), ("omega", ctypes.c_double),
                ("nbottom", ctypes.c_int), ("rcond", ctypes.c_double), ("exact_j", ctypes.c_int)]


class ModelDesc(ctypes.Structure):
    _fields_ = [("ncomp", ctypes.c_int), ("lmax_comp", c_int_p),
                ("inv_cl", ctypes.POINTER(c_double_p)), ("nbands", ctypes.c_int),
                ("bands", ctypes.POINTER(BandDesc)), ("flags", ctypes.c_int)]


_SIGS = {
    "crs_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "crs_last_error": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t]),
    "crs_version": (ctypes.c_char_p, []),
    "crs_grid_healpix": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(vp)]),
    "crs_grid_gauss_legendre": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)]),
    "crs_grid_info": (ctypes.c_int, [vp, c_int_p, c_int64_p]),
    "crs_grid_pixel_centres": (ctypes.c_int, [vp, c_double_p, c_double_p]),
    "crs_grid_weights": (ctypes.c_int, [vp, c_double_p]),
    "crs_grid_destroy": (ctypes.c_int, [vp]),
    "crs_sht_reserve": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp]),
    "sht_synth": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int64, vp,
                                 ctypes.c_int64, vp]),
    "sht_adjoint": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int64, vp,
                                   ctypes.c_int64, vp]),
    "sht_adjoint_noalloc": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int64, vp,
                                           ctypes.c_int64, vp]),
    "crs_autotune_legendre": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp]),
    "crs_legendre_choice": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "crs_model_create": (ctypes.c_int, [ctypes.POINTER(ModelDesc), vp, ctypes.POINTER(vp)]),
    "crs_model_destroy": (ctypes.c_int, [vp]),
    "crs_model_size": (ctypes.c_int, [vp, c_int64_p]),
    "crs_model_alpha2": (ctypes.c_int, [vp, c_double_p]),
    "crs_model_plan_bytes": (ctypes.c_int, [vp, ctypes.c_int, c_int64_p, c_int64_p]),
    "crs_model_set_mixing": (ctypes.c_int, [vp, c_double_p, vp]),
    "crs_model_set_mixing_map": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp, c_double_p, vp]),
    "crs_model_merge_observations": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int), vp]),
    "crs_model_set_mask": (ctypes.c_int, [vp, vp, ctypes.POINTER(ctypes.c_uint8),
                                          ctypes.POINTER(MaskOpts), vp]),
    "crs_model_mask_info": (ctypes.c_int, [vp, c_int_p, c_int_p, ctypes.c_int]),
    "apply_mask_precond": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp]),
    "apply_A": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp]),
    "apply_pinv_precond": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp]),
    "apply_diag_precond": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp]),
    "pcg_solve": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_double,
                                 ctypes.c_int, c_int_p, c_double_p, c_double_p, vp]),
    "build_rhs": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp), vp,
                                 vp, vp]),
    "constrained_realization": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(vp),
                                               ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_double, ctypes.c_int, vp, c_int_p,
                                               c_double_p, vp]),
    "crs_model_project": (ctypes.c_int, [vp, ctypes.c_int, vp, ctypes.POINTER(vp), vp]),
    "apply_prior_inv": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp]),
    "crs_prior_quad": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp, vp]),
    "crs_chi2": (ctypes.c_int, [vp, ctypes.c_int, vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp, vp]),
    "crs_noise_weight": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_double, ctypes.POINTER(vp),
                                        ctypes.POINTER(vp), vp]),
    "apply_dA_dmix": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp, vp]),
    "apply_db_dmix": (ctypes.c_int, [vp, ctypes.c_int, vp, ctypes.POINTER(vp), vp, vp]),
    "crs_batch_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int, vp, ctypes.POINTER(vp)]),
    "crs_batch_destroy": (ctypes.c_int, [vp]),
    "crs_batch_info": (ctypes.c_int, [vp, c_int_p, c_int64_p]),
    "crs_batch_solve": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(ctypes.POINTER(vp)),
                                       ctypes.POINTER(ctypes.c_uint64), ctypes.c_int,
                                       ctypes.c_double, ctypes.c_int, ctypes.POINTER(vp), c_int_p,
                                       c_double_p, ctypes.c_int, vp]),
    "crs_batch_stats": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int)]),
    "crs_batch_set_streams": (ctypes.c_int, [vp, ctypes.c_int]),
    "crs_philox_normals": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_int64, vp, vp]),
    "crs_set_profiling": (ctypes.c_int, [ctypes.c_int]),
    "crs_kernel_stats": (ctypes.c_int, [ctypes.c_char_p, c_int64_p, c_double_p, c_double_p]),
    "crs_kernel_work_counts": (ctypes.c_int, [ctypes.c_char_p, c_double_p]),
    "crs_kernel_stats_reset": (ctypes.c_int, []),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'` "
                "or `python paper_1710_00621_amd/csrc/build.py`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def check(status, allow=()):
    if status == CRS_OK or status in allow:
        return status
    buf = ctypes.create_string_buffer(1024)
    lib().crs_last_error(buf, 1024)
    raise CrsError(status, buf.value.decode(errors="replace"))
