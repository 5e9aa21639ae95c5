"""Helpers of the GPU test modules (no test cases here)."""
import sys

import numpy as np

import oracle


def say(msg: str):
    """Names the case before a GPU step, so a failing run shows where it was."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def gpu_run(q, rho_A, rho_B, tau_A, tau_B, G, steps, *, precision="fp64", kernel=None,
            body_A=0.0, u=None, forcing="shift", tau_minus=None):
    from paper_1112_5547_amd import Lattice
    nz, ny, nx = rho_A.shape
    lat = Lattice(q, nx, ny, nz, tau_A=tau_A, tau_B=tau_B, G=G, precision=precision,
                  body_A=body_A, forcing=forcing, tau_minus=tau_minus)
    if kernel is not None:
        lat.set_kernel(*kernel)
    lat.init(rho_A, rho_B, u)
    lat.step(steps)
    f = lat.get_populations()
    return lat, f


def oracle_run(q, rho_A, rho_B, tau_A, tau_B, G, steps, body_A=0.0, u=None, forcing="shift",
               tau_minus=None):
    f0 = oracle.init(q, rho_A, rho_B, u)
    return oracle.run(f0, tau_A, tau_B, G, steps, body_A=body_A, forcing=forcing,
                      tau_minus=tau_minus)


def maxabs(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max())
