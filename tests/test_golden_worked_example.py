"""The paper's printed worked example (Sec. 4, Tables 1 and 2) against the
definitions of Table 1, fixing two readings of the text:

* tau = 0.55 (Sec. 4 text), not Table 2's 0.5: g^(tau) = tau g / (tau - 1/2)
  prints 1.804 only for 0.55 (and 0.5 would divide by zero);
* kappa = g c_S^4 / 4 and beta = g c_S^2 / 2 with H = 100 / (2 pi) and Re = 1
  reproduce the printed Ch, Pe and Ca.
"""
import json
import math
import os

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    with open(os.path.join(HERE, "golden", "worked_example.json")) as fh:
        return json.load(fh)


def test_g_tau_fixes_tau_reading():
    g = _golden()["sc_parameters"]
    tau, gab = g["tau_text"], g["g_AB"]
    assert abs(tau * gab / (tau - 0.5) - g["g_tau"]) < 5e-4
    assert g["tau_table2_misprint"] - 0.5 == 0.0   # would make g^(tau) singular


def test_table1_definitions_reproduce_table2_groups():
    gold = _golden()
    g = gold["sc_parameters"]
    rho, tau, gab, cs2 = g["rho"], g["tau_text"], g["g_AB"], g["cs2"]
    gt = tau * gab / (tau - 0.5)
    H = 100.0 / (2.0 * math.pi)
    nu = cs2 * (tau - 0.5)
    M = rho * (tau - 0.5)
    kappa = gab * cs2 * cs2 / 4.0
    beta = gab * cs2 / 2.0
    beta_t = gt * cs2 / 2.0
    xi = math.sqrt(kappa / beta)
    U = nu / H                                   # Re = U H / nu = 1
    pe = U * H / (beta_t * M)
    ch = xi / H
    ca = nu * rho * U / math.sqrt(beta * kappa)
    p = gold["phase_field_groups"]
    assert abs(pe - p["Pe"]) / p["Pe"] < 2e-3
    assert abs(ch - p["Ch"]) / p["Ch"] < 3e-3
    assert abs(ca - p["Ca"]) / p["Ca"] < 5e-2    # printed to 2 significant digits


def test_worked_example_values_drive_oracle_run():
    """The oracle run at the golden parameters gives |phi| within 5 % of the
    printed bulk value (the longer run lives in test_oracle_physics)."""
    import numpy as np
    import sc_inputs
    g = _golden()["sc_parameters"]
    fl = sc_inputs.flat_interface(64, 1, 1, rho_total=g["rho"], phi0=1.0)
    f = oracle.init(9, fl.rho_A, fl.rho_B)
    f = oracle.run(f, g["tau_text"], g["tau_text"], g["g_AB"], 40000)
    rho = oracle.observables(f, g["tau_text"], g["tau_text"], g["g_AB"])[0]
    phi = rho[0, 0, 0, 32] - rho[1, 0, 0, 32]
    assert abs(phi - _golden()["bulk_phi"]) < 0.05
