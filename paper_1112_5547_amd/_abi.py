"""ctypes declarations of the C ABI in include/lbm_sc.h (argument marshalling only).

The shared library is built in-tree by ``paper_1112_5547_amd.build``.  Loading
fails loudly when it is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_SC_LIB points the binding at another build of the same library (e.g. one
# compiled with different tile tables); it must export the same symbols.
LIB_PATH = os.environ.get("LBM_SC_LIB") or os.path.join(HERE, "liblbm_sc.so")

LBM_D2Q9, LBM_D3Q19 = 9, 19
LBM_FP64, LBM_FP32_SHIFTED = 0, 1
LBM_FORCING_SHIFT, LBM_FORCING_GUO = 0, 1
LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE = 0, -1, -2, -3
LBM_ESTATE, LBM_ENONFINITE, LBM_EBUDGET, LBM_ETIMEOUT = -4, -5, -6, -7
LBM_ETOOBIG = -8
LBM_BATCH_PER_LATTICE, LBM_BATCH_FUSED, LBM_BATCH_PERSISTENT = 0, 1, 2


class Params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("tau_A", ctypes.c_double), ("tau_B", ctypes.c_double),
        ("G", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("rho_ref_A", ctypes.c_double), ("rho_ref_B", ctypes.c_double),
        ("body_A", ctypes.c_double),
        ("forcing", ctypes.c_int),
        ("tau_minus_A", ctypes.c_double), ("tau_minus_B", ctypes.c_double),
    ]


class Totals(ctypes.Structure):
    _fields_ = [
        ("mass_A", ctypes.c_double), ("mass_B", ctypes.c_double),
        ("mom", ctypes.c_double * 3),
        ("max_u", ctypes.c_double),
        ("ke", ctypes.c_double),
        ("p_in", ctypes.c_double), ("p_out", ctypes.c_double), ("dp", ctypes.c_double),
        ("rhoA_in", ctypes.c_double), ("rhoA_out", ctypes.c_double),
        ("R_eff", ctypes.c_double),
        ("n_in", ctypes.c_double), ("n_out", ctypes.c_double),
        ("n_phi_pos", ctypes.c_double),
        ("n_nonfinite", ctypes.c_double),
        ("step", ctypes.c_longlong),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "mom"}
        d["mom_x"], d["mom_y"], d["mom_z"] = self.mom[0], self.mom[1], self.mom[2]
        return d


# (name, restype, argtypes) of every exported function
_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)
SIGNATURES = [
    ("lbm_sc_params_default", _I, [ctypes.POINTER(Params), _I, _I, _I, _I, _D, _D, _D]),
    ("lbm_sc_bytes_needed", ctypes.c_size_t, [ctypes.POINTER(Params)]),
    ("lbm_sc_create", _I, [ctypes.POINTER(_P), _I, _I, _I, _I, _D, _D, _D]),
    ("lbm_sc_create_ex", _I, [ctypes.POINTER(_P), ctypes.POINTER(Params), _P, _P, ctypes.c_size_t]),
    ("lbm_sc_init", _I, [_P, _DP, _DP, _DP]),
    ("lbm_sc_step", _I, [_P, _I]),
    ("lbm_sc_set_probe", _I, [_P, _D, _D, _D, _D]),
    ("lbm_sc_moments", _I, [_P, _DP, _DP, _DP, ctypes.POINTER(Totals)]),
    ("lbm_sc_get_populations", _I, [_P, _DP]),
    ("lbm_sc_set_populations", _I, [_P, _DP]),
    ("lbm_sc_sync", _I, [_P]),
    ("lbm_sc_time_steps", _I, [_P, _I, ctypes.POINTER(ctypes.c_float)]),
    ("lbm_sc_set_kernel", _I, [_P, _I, _I, _I, _I]),
    ("lbm_sc_get_kernel", _I, [_P, _IP, _IP, _IP, _IP]),
    ("lbm_sc_tile_count", _I, [_I]),
    ("lbm_sc_tile_get", _I, [_I, _I, _IP, _IP]),
    ("lbm_sc_steps_done", ctypes.c_longlong, [_P]),
    ("lbm_sc_get_params", _I, [_P, ctypes.POINTER(Params)]),
    ("lbm_sc_device_buffers", _I, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), _IP]),
    ("lbm_sc_buffer_layout", _I, [_P, ctypes.POINTER(ctypes.c_size_t), _IP]),
    ("lbm_sc_destroy", _I, [_P]),
    ("lbm_sc_strerror", ctypes.c_char_p, [_I]),
    ("lbm_sc_copy_bench", _I, [_P, _P, ctypes.c_size_t, _I, _P, ctypes.POINTER(ctypes.c_float)]),
    ("lbm_batch_create", _I, [ctypes.POINTER(_P), ctypes.c_size_t, _P]),
    ("lbm_batch_add", _I, [_P, _P, ctypes.c_longlong]),
    ("lbm_batch_remove", _I, [_P, _P]),
    ("lbm_batch_run", _I, [_P, _I, _I]),
    ("lbm_batch_run_noalloc", _I, [_P, _I, _I]),
    ("lbm_batch_poll", _I, [_P, ctypes.POINTER(_P), _I, _IP]),
    ("lbm_batch_stats", _I, [_P, _IP, ctypes.POINTER(ctypes.c_size_t), _DP]),
    ("lbm_batch_set_tiles", _I, [_P, _I, _I, _I, _I, _I]),
    ("lbm_batch_set_spin_limit", _I, [_P, ctypes.c_uint]),
    ("lbm_batch_destroy", _I, [_P]),
]

_lib = None


class LbmError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        msg = lib().lbm_sc_strerror(status).decode()
        super().__init__(f"{what}: {msg} (status {status})")


def lib():
    """The loaded library; raises if it has not been built.

    PyTorch bundles its own HIP and HSA runtimes under the same sonames as
    /opt/rocm's.  Importing torch first lets the loader bind this library to
    the runtime torch already mapped, so one process holds one HIP runtime
    (two would both try to own the device).
    """
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with paper_1112_5547_amd.build.build() "
                "(hipcc, gfx950); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int, what: str) -> int:
    if status < 0:
        raise LbmError(status, what)
    return status


def dptr(a):
    """ctypes double* of a C-contiguous float64 numpy array (or None)."""
    if a is None:
        return None
    assert a.dtype.name == "float64" and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)
