"""Python handle of one Shan-Chen lattice (marshalling over the C ABI).

PyTorch provides the device memory (one uint8 arena tensor per lattice) and
the HIP stream the library enqueues on; every step of the method runs in the
library's HIP kernels.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

import numpy as np

from . import _abi
from ._abi import Params, Totals, check, dptr, lib

_PREC = {"fp64": _abi.LBM_FP64, "fp32_shifted": _abi.LBM_FP32_SHIFTED,
         "f64": _abi.LBM_FP64, "f32s": _abi.LBM_FP32_SHIFTED}
_FORCING = {"shift": _abi.LBM_FORCING_SHIFT, "guo": _abi.LBM_FORCING_GUO}


class Lattice:
    """A periodic two-species Shan-Chen lattice on the GPU.

    lattice: 9 (D2Q9, nz = 1) or 19 (D3Q19); tau_B defaults to tau_A;
    precision: "fp64" or "fp32_shifted"; rho_ref: (A, B) reference densities of
    the shifted storage (default: the mean of the initial densities);
    body_A: Kolmogorov forcing amplitude (F_x = rho_s A sin(2 pi y / ny));
    forcing: "shift" (the paper's velocity shift) or "guo" (Guo discrete forcing);
    tau_minus: (tau-_A, tau-_B) relaxation times of the odd moments (two
    relaxation times: viscosity from tau_s, interdiffusion from tau-_s); None
    keeps one relaxation time (BGK).
    """

    def __init__(self, lattice: int, nx: int, ny: int, nz: int = 1, *, tau_A: float = 1.0,
                 tau_B: Optional[float] = None, G: float = 0.0, precision: str = "fp64",
                 rho_ref: Optional[Tuple[float, float]] = None, body_A: float = 0.0,
                 forcing: str = "shift", tau_minus: Optional[Tuple[float, float]] = None,
                 device: Optional[int] = None, use_torch: bool = True):
        L = lib()
        p = Params()
        check(L.lbm_sc_params_default(ctypes.byref(p), lattice, nx, ny, nz, tau_A,
                                      tau_A if tau_B is None else tau_B, G), "params")
        p.precision = _PREC[precision]
        if rho_ref is not None:
            p.rho_ref_A, p.rho_ref_B = float(rho_ref[0]), float(rho_ref[1])
        p.body_A = float(body_A)
        if forcing not in _FORCING:
            raise ValueError(f"forcing must be one of {sorted(_FORCING)}")
        p.forcing = _FORCING[forcing]
        if tau_minus is not None:
            p.tau_minus_A, p.tau_minus_B = float(tau_minus[0]), float(tau_minus[1])
        self.forcing = forcing
        self.tau_minus = tau_minus
        self.params = p
        self.q = lattice
        self.shape = (nz, ny, nx)
        self.n = nx * ny * nz
        self.precision = precision
        self._h = ctypes.c_void_p()
        self._arena = None
        self._stream = None
        nbytes = L.lbm_sc_bytes_needed(ctypes.byref(p))
        if nbytes == 0:
            raise ValueError("invalid lattice parameters")
        self.nbytes = int(nbytes)
        if use_torch:
            import torch
            dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
            with torch.cuda.device(dev):
                self._arena = torch.empty(self.nbytes, dtype=torch.uint8, device=dev)
                self._stream = torch.cuda.Stream(device=dev)
                check(L.lbm_sc_create_ex(ctypes.byref(self._h), ctypes.byref(p),
                                         ctypes.c_void_p(self._stream.cuda_stream),
                                         ctypes.c_void_p(self._arena.data_ptr()),
                                         self.nbytes), "create")
        else:
            check(L.lbm_sc_create_ex(ctypes.byref(self._h), ctypes.byref(p), None, None, 0),
                  "create")

    # -- lifetime --------------------------------------------------------
    def close(self):
        if self._h:
            h, self._h = self._h, ctypes.c_void_p()
            rc = lib().lbm_sc_destroy(h)
            if rc == _abi.LBM_ESTATE:      # still in a batch: nothing was freed
                self._h = h
            check(rc, "destroy")
        self._arena = None
        self._stream = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    # -- state -----------------------------------------------------------
    def init(self, rho_A: np.ndarray, rho_B: np.ndarray, u: Optional[np.ndarray] = None):
        a = np.ascontiguousarray(rho_A, dtype=np.float64).reshape(self.shape)
        b = np.ascontiguousarray(rho_B, dtype=np.float64).reshape(self.shape)
        uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape((3,) + self.shape)
        check(lib().lbm_sc_init(self._h, dptr(a), dptr(b), dptr(uu)), "init")
        return self

    def step(self, n: int = 1):
        check(lib().lbm_sc_step(self._h, int(n)), "step")
        return self

    def sync(self):
        check(lib().lbm_sc_sync(self._h), "sync")

    def time_steps(self, n: int) -> float:
        ms = ctypes.c_float()
        check(lib().lbm_sc_time_steps(self._h, int(n), ctypes.byref(ms)), "time_steps")
        return float(ms.value)

    @property
    def steps_done(self) -> int:
        return int(lib().lbm_sc_steps_done(self._h))

    def set_probe(self, cx: float, cy: float, cz: float, R: float):
        check(lib().lbm_sc_set_probe(self._h, cx, cy, cz, R), "set_probe")

    def moments(self, fields: bool = True, allow_nonfinite: bool = False):
        """(rho_A, rho_B, u_phys, totals) in FP64; fields None when fields=False."""
        T = Totals()
        if fields:
            rA = np.empty(self.shape)
            rB = np.empty(self.shape)
            u = np.empty((3,) + self.shape)
            rc = lib().lbm_sc_moments(self._h, dptr(rA), dptr(rB), dptr(u), ctypes.byref(T))
        else:
            rA = rB = u = None
            rc = lib().lbm_sc_moments(self._h, None, None, None, ctypes.byref(T))
        if not (allow_nonfinite and rc == _abi.LBM_ENONFINITE):
            check(rc, "moments")
        return rA, rB, u, T.as_dict()

    def totals(self, allow_nonfinite: bool = False) -> dict:
        return self.moments(fields=False, allow_nonfinite=allow_nonfinite)[3]

    def get_populations(self) -> np.ndarray:
        f = np.empty((2, self.q) + self.shape)
        check(lib().lbm_sc_get_populations(self._h, dptr(f)), "get_populations")
        return f

    def set_populations(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape((2, self.q) + self.shape)
        check(lib().lbm_sc_set_populations(self._h, dptr(f)), "set_populations")

    # -- kernel configuration ------------------------------------------------
    def set_kernel(self, variant: int = 0, tx: Optional[int] = None, ty: Optional[int] = None,
                   mb: Optional[int] = None):
        v, x, y, m = self.kernel
        check(lib().lbm_sc_set_kernel(self._h, variant, tx or x, ty or y, mb or m), "set_kernel")

    @property
    def kernel(self):
        v, x, y, m = (ctypes.c_int() for _ in range(4))
        check(lib().lbm_sc_get_kernel(self._h, ctypes.byref(v), ctypes.byref(x), ctypes.byref(y),
                                      ctypes.byref(m)), "get_kernel")
        return v.value, x.value, y.value, m.value

    @property
    def buffer_layout(self):
        """(buf0, buf1, current, stride, pitch): device addresses of the two
        population buffers, the one holding the current state, and their
        layout (array (s, i) at element (s Q + i) stride, site (x, y, z) at
        element (z ny + y) pitch + x of it)."""
        b0, b1 = ctypes.c_void_p(), ctypes.c_void_p()
        cur, pitch, stride = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
        check(lib().lbm_sc_device_buffers(self._h, ctypes.byref(b0), ctypes.byref(b1),
                                          ctypes.byref(cur)), "device_buffers")
        check(lib().lbm_sc_buffer_layout(self._h, ctypes.byref(stride), ctypes.byref(pitch)),
              "buffer_layout")
        return b0.value, b1.value, cur.value, stride.value, pitch.value

    @property
    def rho_ref(self):
        p = Params()
        check(lib().lbm_sc_get_params(self._h, ctypes.byref(p)), "get_params")
        return p.rho_ref_A, p.rho_ref_B

    @property
    def stream(self):
        return self._stream


def tiles(lattice: int):
    """Tile shapes (tx, ty) compiled for the lattice type."""
    L = lib()
    out = []
    for k in range(L.lbm_sc_tile_count(lattice)):
        x, y = ctypes.c_int(), ctypes.c_int()
        check(L.lbm_sc_tile_get(lattice, k, ctypes.byref(x), ctypes.byref(y)), "tile_get")
        out.append((x.value, y.value))
    return out


def bytes_needed(lattice: int, nx: int, ny: int, nz: int = 1, precision: str = "fp64") -> int:
    p = Params()
    lib().lbm_sc_params_default(ctypes.byref(p), lattice, nx, ny, nz, 1.0, 1.0, 0.0)
    p.precision = _PREC[precision]
    return int(lib().lbm_sc_bytes_needed(ctypes.byref(p)))


def copy_bench(nbytes: int, reps: int = 10) -> float:
    """Achievable read+write bandwidth (GB/s) of a streaming copy of nbytes."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    s = torch.cuda.Stream()
    ms = ctypes.c_float()
    check(lib().lbm_sc_copy_bench(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                  nbytes, reps, ctypes.c_void_p(s.cuda_stream), ctypes.byref(ms)),
          "copy_bench")
    return 2.0 * nbytes / (ms.value * 1e-3) / 1e9
