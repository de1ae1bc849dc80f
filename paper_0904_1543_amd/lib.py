"""ctypes binding of libwvl (include/wvl.h): same names, argument marshalling only.

Every computation happens in the HIP kernels of libwvl.so.  If the library has
not been built, importing this module raises: there is no fallback path.

torch is imported first so that libwvl resolves its HIP runtime to the one
torch already loaded (one runtime per process; torch's stream handles and
device pointers are then valid in libwvl).
"""

import ctypes
import os

import torch  # noqa: F401  (must be loaded before libwvl, see above)

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libwvl.so")

WVL_OK, WVL_EINVAL, WVL_EUNSUPPORTED, WVL_ENOMEM, WVL_EHIP, WVL_ETIMEOUT, WVL_ENODEV = \
    0, -1, -2, -3, -4, -5, -6
WVL_F64, WVL_F32, WVL_F32C = 0, 1, 2
WVL_SHARED_V, WVL_USE_GRAPH, WVL_PERSISTENT, WVL_AUTOTUNE = 1, 2, 4, 8
WVL_FREE_BC, WVL_SURFACE_BC = 16, 32
(WVL_Q_VARIANT, WVL_Q_GROUP, WVL_Q_PERSISTENT, WVL_Q_XDIV, WVL_Q_PGRID, WVL_Q_TUNE_BEST,
 WVL_Q_FUSED_Z, WVL_Q_PRECOND_FORM) = range(8)
WVL_PRECOND_SEPARATE, WVL_PRECOND_PASSES = 1, 2

STATUS_NAMES = {0: "WVL_OK", -1: "WVL_EINVAL", -2: "WVL_EUNSUPPORTED", -3: "WVL_ENOMEM",
                -4: "WVL_EHIP", -5: "WVL_ETIMEOUT", -6: "WVL_ENODEV"}


class wvl_orbital(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("reserved", ctypes.c_int32),
                ("off", ctypes.c_int64), ("v_off", ctypes.c_int64),
                ("hgrid", ctypes.c_double * 3), ("occ", ctypes.c_double)]


class WvlError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


if not os.path.exists(LIBPATH):
    raise ImportError(f"libwvl.so not built ({LIBPATH}); run __graft_entry__.build()")

_lib = ctypes.CDLL(LIBPATH)

P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
D = ctypes.c_double
DP = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "wvl_create": [ctypes.POINTER(P), ctypes.c_int],
    "wvl_destroy": [P],
    "wvl_plan_create": [P, ctypes.POINTER(wvl_orbital), I32, I32, ctypes.c_uint32,
                        ctypes.POINTER(P)],
    "wvl_plan_destroy": [P],
    "wvl_plan_workspace": [P, ctypes.POINTER(ctypes.c_size_t)],
    "wvl_plan_elements": [P, ctypes.POINTER(I64)],
    "wvl_plan_grid_points": [P, ctypes.POINTER(I64)],
    "wvl_synthesis": [P, P, P, P, P],
    "wvl_analysis": [P, P, P, P, P],
    "wvl_magic_filter": [P, P, P, ctypes.c_int, P, P],
    "wvl_kinetic": [P, P, P, P, P, P],
    "wvl_local_density": [P, P, P, ctypes.c_int, P, P],
    "wvl_local_hpsi": [P, P, P, D, D, P, P, P, P, P, P, P],
    "wvl_overlap": [P, P, P, P, P],
    "wvl_orthonormalize": [P, P, P, P, P, P],
    "wvl_orthonormalize_noalloc": [P, P, P, P, P],
    "wvl_convert": [P, P, I32, P, I32, I64, P],
    "wvl_plan_sync": [P, P],
    "wvl_plan_tuning": [P, ctypes.POINTER(I32), DP, I32],
    "wvl_plan_query": [P, I32, ctypes.POINTER(I64)],
    "wvl_energy_gradient": [P, P, P, D, D, P, P, P],
    "wvl_precondition": [P, P, DP, I32, ctypes.c_uint32, P, P, P, P],
    "wvl_plan_set_regions": [P, ctypes.POINTER(I32), I32, ctypes.POINTER(I32), I32],
    "wvl_plan_compressed_size": [P, ctypes.POINTER(I64), ctypes.POINTER(I64)],
    "wvl_decompress": [P, P, P, P],
    "wvl_compress": [P, P, P, P],
    "wvl_local_hpsi_compressed": [P, P, P, D, D, P, P, P, P, P, P, P],
    "wvl_plan_profile": [P, I32],
    "wvl_plan_profile_read": [P, ctypes.POINTER(I32), DP, I32, ctypes.POINTER(I32)],
}

EXPORTS = list(_SIGS) + ["wvl_last_error", "wvl_version", "wvl_stage_name"]

for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.wvl_last_error.restype = ctypes.c_char_p
_lib.wvl_last_error.argtypes = []
_lib.wvl_version.restype = ctypes.c_char_p
_lib.wvl_version.argtypes = []
_lib.wvl_stage_name.restype = ctypes.c_char_p
_lib.wvl_stage_name.argtypes = [I32]


def wvl_stage_name(stage):
    return _lib.wvl_stage_name(stage).decode()


def wvl_last_error():
    return _lib.wvl_last_error().decode()


def wvl_version():
    return _lib.wvl_version().decode()


def check(code):
    if code != WVL_OK:
        raise WvlError(code, wvl_last_error())
    return code


def raw(name):
    """The ctypes function itself (returns the status code, no checking)."""
    return getattr(_lib, name)


def _mk(name):
    f = getattr(_lib, name)

    def call(*args):
        return check(f(*args))
    call.__name__ = name
    return call


for _name in _SIGS:
    globals()[_name] = _mk(_name)
