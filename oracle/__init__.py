"""CPU oracle of the two-component Shan-Chen BGK lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  The HIP library (``paper_1112_5547_amd``) never
imports, links or executes anything here.  Only the test suite, the package
smoke check and the benchmark's CPU-baseline leg use this package.

Two independent implementations of the same method (Scarbolo et al., Sec. 2.1):

* ``sc_oracle.c`` -- plain C, FP64, loop-per-step, loaded through ctypes
  (``run``, ``collide``, ``stream``, ``observables``, ...);
* ``twin`` -- a NumPy implementation written independently (``np.roll`` push
  streaming, vectorised moments) used to cross-check the C oracle on small
  grids.

The state held between steps is the post-streaming population array
``f[s][i][z][y][x]`` (species A = 0, B = 1), float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_sc.so")
# the same source built with OpenMP: used only to time the oracle on all host cores
_LIB_OMP = os.path.join(_HERE, "liboracle_sc_omp.so")

# totals layout of oracle_observables
TOTAL_KEYS = ("mass_A", "mass_B", "mom_x", "mom_y", "mom_z", "max_u", "p_in", "p_out",
              "dp", "R_eff", "n_phi_pos", "ke", "rhoA_in", "rhoA_out", "n_in", "n_out")

CS2 = 1.0 / 3.0


_CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-D_DEFAULT_SOURCE",
           "-fPIC", "-shared", "-Wall"]


def _stale(path: str) -> bool:
    return not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC)


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc, -O2, no FMA contraction, no fast-math): the
    single-threaded library every check uses, and the same source with OpenMP
    for the all-core timing of the CPU baseline."""
    if force or _stale(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *_CFLAGS, "-Wno-unknown-pragmas", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    if force or _stale(_LIB_OMP):
        tmp = _LIB_OMP + ".tmp"
        subprocess.check_call(["gcc", *_CFLAGS, "-fopenmp", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_OMP)
    return _LIB


_libs = {}


def lib(all_cores: bool = False):
    """The single-threaded oracle library, or its OpenMP build (all_cores)."""
    path = _LIB_OMP if all_cores else _LIB
    if path not in _libs:
        if _stale(path):
            build(force=True)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lp = ctypes.POINTER(ctypes.c_long)
        i, d = ctypes.c_int, ctypes.c_double
        L.oracle_lattice.argtypes = [i, ip, dp]
        L.oracle_feq.argtypes = [i, d, dp, dp]
        L.oracle_init.argtypes = [i, i, i, i, dp, dp, dp, dp]
        L.oracle_moments.argtypes = [i, i, i, i, dp, dp, dp]
        L.oracle_force.argtypes = [i, i, i, i, d, dp, dp]
        L.oracle_collide.argtypes = [i, i, i, i, d, d, d, d, dp, dp, i, d, d]
        L.oracle_stream.argtypes = [i, i, i, i, dp, dp]
        L.oracle_run.argtypes = [i, i, i, i, d, d, d, d, dp, i, i, d, d]
        L.oracle_observables.argtypes = [i, i, i, i, d, d, d, d, dp, dp, dp, dp, dp, dp]
        L.oracle_step_sites.argtypes = [i, i, i, i, d, d, d, d, dp, lp, i, dp, i, d, d]
        for fn in ("oracle_lattice", "oracle_feq", "oracle_init", "oracle_moments",
                   "oracle_force", "oracle_collide", "oracle_stream", "oracle_run",
                   "oracle_observables", "oracle_step_sites"):
            getattr(L, fn).restype = ctypes.c_int
        _libs[path] = L
    return _libs[path]


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


def lattice(q: int):
    """(c[Q,3] int, w[Q] float64) of the oracle's velocity set."""
    c = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q)
    _check(lib().oracle_lattice(q, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _p(w)),
           "lattice")
    return c.astype(np.int64), w


def feq(q: int, rho: float, v: Sequence[float]) -> np.ndarray:
    out = np.zeros(q)
    vv = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(3))
    _check(lib().oracle_feq(q, rho, _p(vv), _p(out)), "feq")
    return out


def _dims(shape):
    nz, ny, nx = shape
    return nx, ny, nz


def init(q: int, rho_A: np.ndarray, rho_B: np.ndarray,
         u: Optional[np.ndarray] = None) -> np.ndarray:
    """f(x, 0) = f^eq(rho_s(x), u(x)); u has shape (3, nz, ny, nx) or is None."""
    rho_A = np.ascontiguousarray(rho_A, dtype=np.float64)
    rho_B = np.ascontiguousarray(rho_B, dtype=np.float64)
    nx, ny, nz = _dims(rho_A.shape)
    f = np.zeros((2, q) + rho_A.shape)
    uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
    _check(lib().oracle_init(q, nx, ny, nz, _p(rho_A), _p(rho_B), _p(uu), _p(f)), "init")
    return f


def moments(f: np.ndarray):
    q = f.shape[1]
    nx, ny, nz = _dims(f.shape[2:])
    rho = np.zeros((2,) + f.shape[2:])
    j = np.zeros((2, 3) + f.shape[2:])
    _check(lib().oracle_moments(q, nx, ny, nz, _p(np.ascontiguousarray(f)), _p(rho), _p(j)),
           "moments")
    return rho, j


def force(q: int, G: float, rho: np.ndarray) -> np.ndarray:
    """F[s, a, z, y, x] from rho[s, z, y, x] (eq. FORCE with psi = rho)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    nx, ny, nz = _dims(rho.shape[1:])
    F = np.zeros((2, 3) + rho.shape[1:])
    _check(lib().oracle_force(q, nx, ny, nz, G, _p(rho), _p(F)), "force")
    return F


FORCING = {"shift": 0, "guo": 1}


def _forcing(name: str) -> int:
    if name not in FORCING:
        raise ValueError(f"forcing must be one of {sorted(FORCING)}")
    return FORCING[name]


def _taum(tau_minus) -> tuple:
    """(tau-_A, tau-_B); None or values <= 0 mean "equal to tau_s" (BGK)."""
    if tau_minus is None:
        return 0.0, 0.0
    return float(tau_minus[0]), float(tau_minus[1])


def collide(f: np.ndarray, tau_A: float, tau_B: float, G: float, body_A: float = 0.0,
            forcing: str = "shift", tau_minus=None):
    """One collision of both species; forcing "shift" is the paper's velocity
    shift (Sec. 2.1), "guo" the discrete forcing it cites (Sec. 2.3);
    tau_minus = (tau-_A, tau-_B) relaxes the odd moments separately (two
    relaxation times)."""
    q = f.shape[1]
    nx, ny, nz = _dims(f.shape[2:])
    f = np.ascontiguousarray(f)
    out = np.zeros_like(f)
    _check(lib().oracle_collide(q, nx, ny, nz, tau_A, tau_B, G, body_A, _p(f), _p(out),
                                _forcing(forcing), *_taum(tau_minus)), "collide")
    return out


def stream(fpost: np.ndarray) -> np.ndarray:
    q = fpost.shape[1]
    nx, ny, nz = _dims(fpost.shape[2:])
    fpost = np.ascontiguousarray(fpost)
    out = np.zeros_like(fpost)
    _check(lib().oracle_stream(q, nx, ny, nz, _p(fpost), _p(out)), "stream")
    return out


def run(f: np.ndarray, tau_A: float, tau_B: float, G: float, steps: int,
        body_A: float = 0.0, forcing: str = "shift", tau_minus=None,
        all_cores: bool = False) -> np.ndarray:
    """``steps`` full collide+stream steps; returns a new array.  all_cores runs
    the OpenMP build of the same source (same result bit for bit; for timing)."""
    q = f.shape[1]
    nx, ny, nz = _dims(f.shape[2:])
    g = np.array(f, dtype=np.float64, order="C", copy=True)
    _check(lib(all_cores).oracle_run(q, nx, ny, nz, tau_A, tau_B, G, body_A, _p(g), steps,
                            _forcing(forcing), *_taum(tau_minus)), "run")
    return g


def observables(f: np.ndarray, tau_A: float, tau_B: float, G: float, probe=None,
                body_A: float = 0.0):
    """(rho[2,...], u_phys[3,...], p[...], totals dict) of the state f."""
    q = f.shape[1]
    shp = f.shape[2:]
    nx, ny, nz = _dims(shp)
    rho = np.zeros((2,) + shp)
    u = np.zeros((3,) + shp)
    p = np.zeros(shp)
    T = np.zeros(len(TOTAL_KEYS))
    pr = None if probe is None else np.ascontiguousarray(np.asarray(probe, dtype=np.float64))
    _check(lib().oracle_observables(q, nx, ny, nz, tau_A, tau_B, G, body_A,
                                    _p(np.ascontiguousarray(f)), _p(pr), _p(rho), _p(u),
                                    _p(p), _p(T)), "observables")
    return rho, u, p, dict(zip(TOTAL_KEYS, T.tolist()))


def step_sites(f: np.ndarray, tau_A: float, tau_B: float, G: float, sites: np.ndarray,
               body_A: float = 0.0, forcing: str = "shift", tau_minus=None) -> np.ndarray:
    """Populations after one step at the given flat site indices: out[k, s, i]."""
    q = f.shape[1]
    nx, ny, nz = _dims(f.shape[2:])
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.zeros((len(sites), 2, q))
    _check(lib().oracle_step_sites(q, nx, ny, nz, tau_A, tau_B, G, body_A,
                                   _p(np.ascontiguousarray(f)),
                                   sites.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                                   len(sites), _p(out), _forcing(forcing), *_taum(tau_minus)),
           "step_sites")
    return out
