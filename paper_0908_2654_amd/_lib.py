"""ctypes binding of librh.so (the C ABI declared in include/rh.h).

Argument marshalling only.  Importing this module loads the library and
raises ImportError if it has not been built: there is no fallback path.
"""
import ctypes
import os

# PyTorch ships its own HIP runtime.  Load it before librh.so so the library
# binds to that same runtime (one process, one runtime): loaded the other way
# round the library gets a second runtime that does not see torch's device
# memory or, on some boxes, any device at all.
import torch  # noqa: F401,E402

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librh.so")

KERNEL_CLASSES = ["step_setup", "local_solve", "residual_schur", "finalize", "rbgs_fine",
                  "mg_residual_fine", "restrict_fine", "prolong_fine", "coarse_levels",
                  "pcg_direction", "pcg_update", "pcg_precond", "defect_update", "cast",
                  "rbgs_fine_colour", "rbgs_fine_dots", "advect", "advect_courant",
                  "block_relax", "block_inverse",
                  # multigroup step only
                  "local_groups", "coupled_residual", "krylov"]

RH_OK, RH_EINVAL, RH_ENOMEM, RH_EHIP, RH_ENONFINITE, RH_ENEWTON, RH_ELINEAR = range(7)
STATUS_NAMES = {0: "RH_OK", 1: "RH_EINVAL", 2: "RH_ENOMEM", 3: "RH_EHIP", 4: "RH_ENONFINITE",
                5: "RH_ENEWTON", 6: "RH_ELINEAR"}

_i32 = ctypes.c_int32
_f64 = ctypes.c_double
_vp = ctypes.c_void_p


class RhParams(ctypes.Structure):
    _fields_ = [
        ("nx", _i32), ("ny", _i32), ("nz", _i32),
        ("bc", _i32 * 6),
        ("box_comoving_cm", _f64),
        ("isothermal", _i32), ("spectrum", _i32),
        ("T_iso_K", _f64), ("T_bb_K", _f64), ("hnu0_eV", _f64), ("sigma0_cm2", _f64),
        ("rates", _i32), ("cooling_mask", _i32),
        ("alphaB_const", _f64),
        ("cosmology", _i32), ("precision", _i32),
        ("hubble_h", _f64), ("Omega_m", _f64), ("Omega_L", _f64),
        ("theta", _f64), ("E_floor", _f64), ("R_min", _f64), ("gamma", _f64),
        ("newton_tol", _f64),
        ("newton_max_it", _i32), ("ls_max_cuts", _i32),
        ("lin_forcing", _f64),
        ("lin_max_it", _i32), ("mg_pre", _i32), ("mg_post", _i32), ("mg_coarse_max", _i32),
        ("krylov", _i32), ("smoother", _i32),
        ("mg_block_radius", _i32), ("mg_block_levels", _i32), ("mg_block_max", _i32),
    ]


class RhStepStats(ctypes.Structure):
    _fields_ = [
        ("newton_its", _i32), ("lin_its_total", _i32), ("ls_cuts", _i32),
        ("local_its_max", _i32),
        ("res0", _f64), ("res_final", _f64), ("lin_res_max", _f64),
        ("t_ms", _f64 * 8),
        ("lin_cap_hits", _i32), ("lin_its_max", _i32), ("source_boxes", _i32),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "t_ms"}
        d["t_ms"] = list(self.t_ms)
        return d


class RhAdvanceStats(ctypes.Structure):
    _fields_ = [
        ("steps", _i32), ("rejected", _i32), ("newton_its", _i32), ("lin_its_total", _i32),
        ("dt_min", _f64), ("dt_max", _f64), ("dt_next", _f64), ("change_max", _f64),
        ("change_last", _f64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RhAdvectStats(ctypes.Structure):
    _fields_ = [("substeps", _i32), ("courant", _f64), ("courant_substep", _f64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# exported symbols and their signatures (name -> (restype, argtypes))
_PP = ctypes.POINTER(RhParams)
_SP = ctypes.POINTER(RhStepStats)
MAX_GROUPS = 4


class RhMultigroupParams(ctypes.Structure):
    _fields_ = [
        ("groups", _i32), ("reserved", _i32),
        ("edge_eV", _f64 * MAX_GROUPS),
        ("y_he", _f64), ("sigma_power", _f64),
    ]


_MP = ctypes.POINTER(RhMultigroupParams)

SIGNATURES = {
    "rh_default_params": (None, [_PP]),
    "rh_workspace_bytes": (ctypes.c_size_t, [_PP]),
    "rh_setup": (_i32, [_PP, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    "rh_implicit_step": (_i32, [_vp, _f64, _f64, _vp, _vp, _vp, _vp, _vp, _SP]),
    "rh_adjoint_step": (_i32, [_vp, _f64, _f64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                               _vp, _vp, _vp, _vp, _vp, _SP]),
    "rh_advance": (_i32, [_vp, _f64, _f64, _f64, _f64, _f64, _vp, _vp, _vp, _vp, _vp,
                          ctypes.POINTER(RhAdvanceStats), ctypes.POINTER(_f64)]),
    "rh_advect": (_i32, [_vp, _f64, _f64, _vp, _vp, _vp, _f64, _vp, _vp, _vp, _vp,
                         ctypes.POINTER(RhAdvectStats)]),
    "rh_residual": (_i32, [_vp, _f64, _f64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                           _vp, _vp, _vp, ctypes.POINTER(_f64)]),
    "rh_residual_noalloc": (_i32, [_PP, _vp, _f64, _f64, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                   _vp, _vp, _vp, _vp, ctypes.POINTER(_f64)]),
    "rh_schur_solve": (_i32, [_vp, _f64, _f64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                              _vp, _vp, _f64, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_f64)]),
    "rh_schur_operator": (_i32, [_vp, _f64, _f64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                 _vp, _vp, _vp, _vp]),
    "rh_initial_state": (_i32, [_vp, _vp, _f64, _f64, _f64, _vp, _vp, _vp]),
    "rh_source_field": (_i32, [_vp, _vp, _vp]),
    "rh_get_constants": (_i32, [_vp, ctypes.POINTER(_f64), _i32]),
    "rh_cosmology_at": (_i32, [_PP, _f64, ctypes.POINTER(_f64), ctypes.POINTER(_f64)]),
    "rh_cosmic_time": (_i32, [_PP, _f64, ctypes.POINTER(_f64)]),
    "rh_set_kernel_timing": (_i32, [_vp, _i32]),
    "rh_get_kernel_timing": (_i32, [_vp, ctypes.POINTER(_f64), ctypes.POINTER(ctypes.c_int64),
                                    _i32, _i32]),
    "rh_last_error": (ctypes.c_char_p, [_vp]),
    "rh_destroy": (None, [_vp]),
    "rh_multigroup_constants": (_i32, [_PP, _MP, ctypes.POINTER(_f64), _i32]),
    "rh_multigroup_workspace_bytes": (ctypes.c_size_t, [_PP, _MP]),
    "rh_multigroup_setup": (_i32, [_PP, _MP, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    "rh_multigroup_initial_state": (_i32, [_vp, _vp, _f64, _f64, _f64, _vp, _vp, _vp]),
    "rh_multigroup_step": (_i32, [_vp, _f64, _f64, _vp, _vp, _vp, _vp, _vp, _SP]),
    "rh_multigroup_residual": (_i32, [_vp, _f64, _f64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                      _vp, _vp, _vp, ctypes.POINTER(_f64)]),
    "rh_multigroup_set_kernel_timing": (_i32, [_vp, _i32]),
    "rh_multigroup_get_kernel_timing": (_i32, [_vp, ctypes.POINTER(_f64),
                                                ctypes.POINTER(ctypes.c_int64), _i32, _i32]),
    "rh_multigroup_last_error": (ctypes.c_char_p, [_vp]),
    "rh_multigroup_destroy": (None, [_vp]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_0908_2654_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


class RhError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status, handle=None):
    if status != RH_OK:
        msg = lib.rh_last_error(handle)
        raise RhError(status, msg.decode() if msg else "")


def check_multigroup(status, handle=None):
    if status != RH_OK:
        msg = lib.rh_multigroup_last_error(handle)
        raise RhError(status, msg.decode() if msg else "")


def default_params() -> RhParams:
    p = RhParams()
    lib.rh_default_params(ctypes.byref(p))
    return p
