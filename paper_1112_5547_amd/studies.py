"""Precision and physics studies of the GPU step (FP64 against FP32 shifted).

* ``spinodal_study``: spinodal decomposition from rho_A = rho_B = 0.5 with
  seeded noise; every ``every`` steps it records the per-species mass drift
  and the domain length of phi = rho_A - rho_B from the structure factor
  S(k) = |FFT(phi - <phi>)|^2: l = 2 pi sum_k S / sum_k |k| S (first moment).
  Pointwise fields of the two precisions diverge once the noise has been
  amplified, so the comparison is statistical.
* ``drop_study``: a static drop; per-species mass, spurious max |u_phys|,
  Laplace pressure Delta p and R_eff in both precisions.

Fields are copied to the host only at the checkpoints; S(k) is evaluated
there with numpy.fft (a diagnostic, not part of the step).
"""
from __future__ import annotations

import time
from typing import Dict, List

import numpy as np

from .lattice import Lattice


def domain_length(phi: np.ndarray) -> float:
    """First-moment domain length of a periodic field (site units)."""
    d = phi - phi.mean()
    S = np.abs(np.fft.fftn(d)) ** 2
    ks = [2 * np.pi * np.fft.fftfreq(n) for n in phi.shape]
    grids = np.meshgrid(*ks, indexing="ij")
    kmag = np.sqrt(sum(g * g for g in grids))
    S.flat[0] = 0.0
    return float(2 * np.pi * S.sum() / (kmag * S).sum())


def spinodal_study(L: int = 256, steps: int = 5000, every: int = 500, *, G: float = 1.6,
                   tau: float = 1.0, seed: int = 3, q: int = 19,
                   precisions=("fp64", "fp32_shifted"), tuned: bool = True) -> Dict[str, List[dict]]:
    import sc_inputs
    from . import autotune
    shape = (L, L, L) if q == 19 else (1, L, L)
    nz, ny, nx = shape
    fl = sc_inputs.spinodal(nx, ny, nz, seed=seed)
    out: Dict[str, List[dict]] = {}
    for prec in precisions:
        lat = Lattice(q, nx, ny, nz, tau_A=tau, G=G, precision=prec)
        if tuned:
            autotune.apply(lat)
        lat.init(fl.rho_A, fl.rho_B)
        rows = []
        _, _, _, T0 = lat.moments(fields=False)
        t_gpu = 0.0
        for k in range(0, steps + 1, every):
            if k > 0:
                t_gpu += lat.time_steps(every) * 1e-3
            rA, rB, _, T = lat.moments(fields=True)
            rows.append({"step": k,
                         "mass_drift_A": (T["mass_A"] - T0["mass_A"]) / T0["mass_A"],
                         "mass_drift_B": (T["mass_B"] - T0["mass_B"]) / T0["mass_B"],
                         "mom": max(abs(T["mom_x"]), abs(T["mom_y"]), abs(T["mom_z"])),
                         "domain_length": domain_length(rA - rB),
                         "max_u": T["max_u"], "n_nonfinite": T["n_nonfinite"],
                         "gpu_seconds": t_gpu})
        lat.close()
        out[prec] = rows
    return out


def drop_study(L: int = 128, steps: int = 1000, *, R: float = 24.0, G: float = 1.3,
               tau: float = 1.0, seed: int = 2, q: int = 19,
               precisions=("fp64", "fp32_shifted")) -> Dict[str, dict]:
    import sc_inputs
    nz = L if q == 19 else 1
    fl = sc_inputs.drop(L, L, nz, radius=R, seed=seed)
    out = {}
    for prec in precisions:
        lat = Lattice(q, L, L, nz, tau_A=tau, G=G, precision=prec)
        lat.init(fl.rho_A, fl.rho_B)
        lat.set_probe(*fl.centre, R)
        _, _, _, T0 = lat.moments(fields=False)
        lat.step(steps)
        rA, rB, u, T = lat.moments()
        out[prec] = {"totals": T, "T0": T0, "rho_A": rA, "u": u}
        lat.close()
    return out


def compare_drop(res: Dict[str, dict]) -> dict:
    a, b = res["fp64"], res["fp32_shifted"]
    ta, tb = a["totals"], b["totals"]
    return {
        "max_abs_rho_A": float(np.abs(a["rho_A"] - b["rho_A"]).max()),
        "max_u_fp64": ta["max_u"], "max_u_fp32": tb["max_u"],
        "max_u_rel": abs(tb["max_u"] - ta["max_u"]) / ta["max_u"],
        "dp_fp64": ta["dp"], "dp_fp32": tb["dp"], "dp_rel": abs(tb["dp"] - ta["dp"]) / abs(ta["dp"]),
        "R_eff_fp64": ta["R_eff"], "R_eff_fp32": tb["R_eff"],
        "mass_drift_A_fp64": (ta["mass_A"] - a["T0"]["mass_A"]) / a["T0"]["mass_A"],
        "mass_drift_A_fp32": (tb["mass_A"] - b["T0"]["mass_A"]) / b["T0"]["mass_A"],
    }


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["spinodal", "drop"])
    ap.add_argument("--L", type=int, default=None)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--every", type=int, default=500)
    a = ap.parse_args()
    t0 = time.time()
    if a.study == "spinodal":
        r = spinodal_study(L=a.L or 256, steps=a.steps or 5000, every=a.every)
        for prec, rows in r.items():
            for row in rows:
                print(json.dumps({"precision": prec, **row}), flush=True)
        l64, l32 = r["fp64"][-1]["domain_length"], r["fp32_shifted"][-1]["domain_length"]
        print(json.dumps({"final_rel_domain_length_diff": abs(l32 - l64) / l64,
                          "wall_s": time.time() - t0}))
    else:
        r = drop_study(L=a.L or 128, steps=a.steps or 1000)
        print(json.dumps(compare_drop(r)))
