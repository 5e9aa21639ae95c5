"""Precision and physics studies of the GPU step (FP64 against FP32 shifted).

* ``spinodal_study``: spinodal decomposition from rho_A = rho_B = 0.5 with
  seeded noise; every ``every`` steps it records the per-species mass drift
  and the domain length of phi = rho_A - rho_B from the structure factor
  S(k) = |FFT(phi - <phi>)|^2: l = 2 pi sum_k S / sum_k |k| S (first moment).
  Pointwise fields of the two precisions diverge once the noise has been
  amplified, so the comparison is statistical.
* ``drop_study``: a static drop; per-species mass, spurious max |u_phys|,
  Laplace pressure Delta p and R_eff in both precisions.
* ``paper_drop_kolmogorov``: the paper's own two-phase test (Sec. 4): a D2Q9
  drop on a periodic 100 x 100 grid with tau = 0.55, rho = 1.4, g_AB = 0.164
  and R = L/4 is run to a steady state (Sec. 4.1: surface tension
  sigma(t) = R [P_i - P_o], spurious currents, bulk order parameter), then
  the Kolmogorov force F_x = rho A sin(2 pi y / L_y), A = 1e-6, is switched on
  (Sec. 4.2: total kinetic energy and the leakage L(t) = M(t) / M_0, M the
  number of nodes with phi >= 0) until the flow is steady again.

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


def paper_drop_kolmogorov(precision: str = "fp64", *, L: int = 100, steps_static: int = 40000,
                          steps_forced: int = 80000, every: int = 1000, A: float = 1e-6,
                          tau: float = 0.55, rho: float = 1.4, G: float = 0.164) -> dict:
    """The paper's static drop and its deformation under Kolmogorov flow.

    The drop starts as a tanh profile of phi = +-1 (rho_A = (rho + phi) / 2),
    at rest, radius L/4.  The forced phase continues from the settled state:
    its populations are moved to a lattice created with the body force (same
    reference densities, so the FP32 shifted storage is carried over
    exactly).  Returns the time series of both phases."""
    import sc_inputs
    R = L / 4.0
    fl = sc_inputs.drop(L, L, 1, radius=R, rho_in=(rho + 1.0) / 2.0, rho_out=(rho - 1.0) / 2.0,
                        width=2.0, noise=0.0)
    cx, cy, cz = fl.centre

    def row(lat, k):
        rA, rB, u, T = lat.moments(fields=True, allow_nonfinite=True)
        phi = rA - rB
        return {"step": k, "sigma": T["R_eff"] * T["dp"], "dp": T["dp"], "R_eff": T["R_eff"],
                "max_u": T["max_u"], "ke": T["ke"], "n_phi_pos": T["n_phi_pos"],
                "phi_in": float(phi[0, int(cy), int(cx)]), "phi_out": float(phi[0, 0, 0]),
                "mass_A": T["mass_A"], "n_nonfinite": T["n_nonfinite"]}

    lat = Lattice(9, L, L, 1, tau_A=tau, G=G, precision=precision)
    lat.init(fl.rho_A, fl.rho_B)
    lat.set_probe(cx, cy, cz, R)
    static = [row(lat, 0)]
    for k in range(every, steps_static + 1, every):
        lat.step(every)
        static.append(row(lat, k))
    f = lat.get_populations()
    ref = lat.rho_ref
    lat.close()

    lat = Lattice(9, L, L, 1, tau_A=tau, G=G, precision=precision, rho_ref=ref, body_A=A)
    lat.set_populations(f)
    lat.set_probe(cx, cy, cz, R)
    forced = [row(lat, 0)]
    for k in range(every, steps_forced + 1, every):
        lat.step(every)
        forced.append(row(lat, k))
    lat.close()
    m0 = forced[0]["n_phi_pos"]
    for r in forced:
        r["leakage"] = r["n_phi_pos"] / m0
    nu = (tau - 0.5) / 3.0
    k = 2.0 * np.pi / L
    return {"static": static, "forced": forced,
            # single-phase Kolmogorov flow at the same forcing: u = A / (nu k^2) sin(k y),
            # sum_x |u|^2 = N (A / (nu k^2))^2 / 2
            "ke_single_phase": L * L * (A / (nu * k * k)) ** 2 / 2.0}


def laplace_study(q: int, L: int, radii, steps: int, *, tau: float = 1.0, G: float = 1.3,
                  rho_in: float = 0.96634, rho_out: float = 0.10221,
                  precision: str = "fp64") -> dict:
    """Static drops of several radii (Sec. 4.1, sigma = R [P_i - P_o] in 2D,
    Delta p = 2 sigma / R in 3D).  Each drop starts from a tanh profile of the
    coexistence densities of a flat interface at (tau, G), runs `steps` steps,
    and gives (R_eff, Delta p).  Fits Delta p = c / R_eff + b by least squares:
    sigma = c (2D) or c / 2 (3D), with r^2 and the intercept b."""
    import sc_inputs
    rows = []
    for R in radii:
        nz = L if q == 19 else 1
        fl = sc_inputs.drop(L, L, nz, radius=R, rho_in=rho_in, rho_out=rho_out, width=1.0,
                            noise=0.0)
        lat = Lattice(q, L, L, nz, tau_A=tau, G=G, precision=precision)
        from . import autotune
        autotune.apply(lat)
        lat.init(fl.rho_A, fl.rho_B)
        lat.set_probe(*fl.centre, R)
        lat.step(steps)
        T = lat.totals()
        lat.close()
        rows.append({"R": R, "R_eff": T["R_eff"], "dp": T["dp"], "max_u": T["max_u"]})
    x = np.array([1.0 / r["R_eff"] for r in rows])
    y = np.array([r["dp"] for r in rows])
    Amat = np.vstack([x, np.ones_like(x)]).T
    (c, b), *_ = np.linalg.lstsq(Amat, y, rcond=None)
    fit = Amat @ np.array([c, b])
    r2 = 1.0 - ((y - fit) ** 2).sum() / ((y - y.mean()) ** 2).sum()
    return {"rows": rows, "sigma": c / (2.0 if q == 19 else 1.0), "intercept": b, "r2": r2,
            "max_dp": float(y.max())}


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
    ap.add_argument("study", choices=["spinodal", "drop", "paper", "laplace"])
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
    elif a.study == "drop":
        r = drop_study(L=a.L or 128, steps=a.steps or 1000)
        print(json.dumps(compare_drop(r)))
    elif a.study == "laplace":
        r2d = laplace_study(9, 128, [10, 14, 18, 22, 26, 30], a.steps or 20000)
        r3d = laplace_study(19, 128, [12, 16, 20, 24, 28], 4000)
        print(json.dumps({"2d": r2d, "3d": r3d,
                          "sigma_rel_diff": abs(r3d["sigma"] - r2d["sigma"]) / r2d["sigma"],
                          "wall_s": time.time() - t0}))
    else:
        for prec in ("fp64", "fp32_shifted"):
            r = paper_drop_kolmogorov(prec, every=a.every)
            for phase in ("static", "forced"):
                for row in r[phase]:
                    print(json.dumps({"precision": prec, "phase": phase, **row}), flush=True)
            print(json.dumps({"precision": prec, "ke_single_phase": r["ke_single_phase"],
                              "wall_s": time.time() - t0}), flush=True)
