"""Linearised Shan-Chen BGK update in Fourier space (test helper).

An independent derivation, used to pin the oracle: about a uniform state
rho_A0, rho_B0 at rest, a perturbation f = f0 + eps Re[fhat e^{i k.x}] evolves
to first order in eps as fhat(t+1) = M(k) fhat(t), with M built here from the
Sec. 2.1 definitions taken one by one:

  drho_s   = sum_i fhat_is                 dj_s = sum_i fhat_is c_i
  dgath_s  = sum_i w_i c_i e^{i k.c_i} drho_s'          (force gather of FORCE)
  dF_s     = -G rho_s0 dgath_s             (the base gather vanishes)
  du       = sum_s dj_s / tau_s / sum_s rho_s0 / tau_s
  dv_s     = du + tau_s dF_s / rho_s0
  dfeq_is  = w_i (drho_s + rho_s0 c_i.dv_s / c_S^2)
  df*_is   = (1 - 1/tau_s) fhat_is + dfeq_is / tau_s
  stream   : fhat_is <- e^{-i k.c_i} df*_is

The velocity set is built from the speed-class rule, not from either oracle.
"""
from __future__ import annotations

import numpy as np

CS2 = 1.0 / 3.0

_ORDER = {
    9: [(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0),
        (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0)],
    19: [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
         (1, 1, 0), (-1, -1, 0), (1, 0, 1), (-1, 0, -1), (0, 1, 1), (0, -1, -1),
         (1, -1, 0), (-1, 1, 0), (1, 0, -1), (-1, 0, 1), (0, 1, -1), (0, -1, 1)],
}
_W = {9: {0: 4 / 9, 1: 1 / 9, 2: 1 / 36}, 19: {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}}


def vset(q):
    c = np.array(_ORDER[q], dtype=np.float64)
    w = np.array([_W[q][int(round((ci * ci).sum()))] for ci in c])
    return c, w


def update_matrix(q: int, k, rho_A0: float, rho_B0: float, tau_A: float, tau_B: float,
                  G: float, forcing: str = "shift", tau_minus=None) -> np.ndarray:
    """The 2Q x 2Q complex matrix M(k) acting on fhat[s*Q + i].

    forcing "guo" linearises the discrete forcing instead of the velocity
    shift: du = sum_s (dj_s + dF_s / 2) / tau_s / sum_s rho_s0 / tau_s, the
    equilibrium at du for every species, plus the source
    (1 - 1/(2 tau_s)) w_i c_i.dF_s / c_S^2 (its terms in u vanish at rest).

    tau_minus = (tm_A, tm_B) relaxes the odd part of each species' deviation
    from equilibrium with tm_s (two relaxation times): the collision acts on
    d = fhat - dfeq as d - P+ d / tau_s - P- d / tm_s, P+- the projections on
    the parts even / odd under c_i -> -c_i; the momentum weights, the force
    shift and the source (all odd) take tm_s."""
    c, w = vset(q)
    k = np.asarray(k, dtype=np.float64)
    phase = np.exp(1j * (c @ k))                       # e^{i k.c_i}
    rho0 = np.array([rho_A0, rho_B0])
    tau = np.array([tau_A, tau_B])
    tm = tau if tau_minus is None else np.array(tau_minus, dtype=np.float64)
    # projections on the even / odd parts under velocity reversal
    rev = np.array([[1.0 if np.all(c[a] == -c[b]) else 0.0 for b in range(q)] for a in range(q)])
    Pe, Po = 0.5 * (np.eye(q) + rev), 0.5 * (np.eye(q) - rev)
    n = 2 * q
    M = np.zeros((n, n), dtype=complex)
    gvec = (w[:, None] * c * phase[:, None]).sum(0)    # sum_i w_i c_i e^{ik.c_i}
    for col in range(n):
        fh = np.zeros((2, q), dtype=complex)
        fh[col // q, col % q] = 1.0
        drho = fh.sum(1)
        dj = fh @ c                                     # [s, 3]
        dgath = np.array([gvec * drho[1], gvec * drho[0]])
        dF = -G * rho0[:, None] * dgath
        out = np.zeros((2, q), dtype=complex)
        if forcing == "guo":
            du = ((dj + 0.5 * dF) / tm[:, None]).sum(0) / (rho0 / tm).sum()
            for s in range(2):
                dfeq = w * (drho[s] + rho0[s] * (c @ du) / CS2)
                dsrc = (1.0 - 0.5 / tm[s]) * w * (c @ dF[s]) / CS2
                d = fh[s] - dfeq
                dfs = fh[s] - Pe @ d / tau[s] - Po @ d / tm[s] + dsrc
                out[s] = np.conj(phase) * dfs
            M[:, col] = out.reshape(-1)
            continue
        du = (dj / tm[:, None]).sum(0) / (rho0 / tm).sum()
        for s in range(2):
            dv = du + tm[s] * dF[s] / rho0[s]
            dfeq = w * (drho[s] + rho0[s] * (c @ dv) / CS2)
            d = fh[s] - dfeq
            dfs = fh[s] - Pe @ d / tau[s] - Po @ d / tm[s]
            out[s] = np.conj(phase) * dfs
        M[:, col] = out.reshape(-1)
    return M


def phi_mode_rate(q, k, rho, tau, G, forcing: str = "shift", tau_minus=None):
    """Growth rate log(lambda) of the order-parameter mode at wavevector k.

    Base state rho_A0 = rho_B0 = rho/2; the phi mode is the eigenvector whose
    density perturbation is antisymmetric (drho_A = -drho_B) with the
    eigenvalue closest to 1.
    """
    M = update_matrix(q, k, rho / 2, rho / 2, tau, tau, G, forcing,
                      None if tau_minus is None else (tau_minus, tau_minus))
    lam, vec = np.linalg.eig(M)
    best = None
    for j in range(len(lam)):
        v = vec[:, j].reshape(2, q)
        dA, dB = v[0].sum(), v[1].sum()
        if abs(dA - dB) < 1e-8:
            continue
        if abs(dA + dB) > 1e-6 * abs(dA - dB):
            continue
        if best is None or abs(lam[j] - 1) < abs(lam[best] - 1):
            best = j
    return np.log(lam[best])


def paper_phi_rate(k: float, rho: float, tau: float, G: float, coupling: str = "g_tau") -> float:
    """Continuum growth rate of a small phi mode from the paper's SC limit.

    Sec. 2.1: d phi/dt = div(M grad mu) with M = rho (tau - 1/2) at phi = 0 and
    mu^(tau) linearised about phi = 0:
      mu ~ (c_S^2 / rho) phi - (g^(tau)/2) c_S^2 phi - (g^(tau)/4) c_S^4 lap(phi),
    g^(tau) = tau G / (tau - 1/2) (coupling "g_tau"; "g" puts the bare G in its
    place, the limit the paper expects once the discrete forcing is cured).
    For phi ~ e^{ikx}:
      omega = -M k^2 [c_S^2/rho - g^(tau) c_S^2/2 + g^(tau) c_S^4 k^2 / 4].
    """
    gt = tau * G / (tau - 0.5) if coupling == "g_tau" else G
    M = rho * (tau - 0.5)
    return -M * k * k * (CS2 / rho - gt * CS2 / 2 + gt * CS2 * CS2 * k * k / 4)
