"""Independent NumPy implementation of the Shan-Chen BGK step (Sec. 2.1).

TEST INFRASTRUCTURE ONLY: a second, differently written oracle used to
cross-check the C oracle on small grids.  It shares nothing with the C file
except the export order of the velocities (a documented convention):

* the weights are not tabulated but derived from the speed class |c|^2, using
  the standard D2Q9 / D3Q19 values that meet the paper's normalisation
  (sum_i w_i c_ia c_ib = c_S^2 delta_ab, fourth-order isotropy, c_S^2 = 1/3);
* streaming is a push with ``np.roll`` instead of the C oracle's index loops;
* moments and the force gather are vectorised over the whole lattice.

Arrays: f[s, i, z, y, x], float64.
"""
from __future__ import annotations

import numpy as np

CS2 = 1.0 / 3.0

# Export order of the library / oracle velocity sets (a convention, not data).
ORDER = {
    9: [(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0),
        (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0)],
    19: [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
         (1, 1, 0), (-1, -1, 0), (1, 0, 1), (-1, 0, -1), (0, 1, 1), (0, -1, -1),
         (1, -1, 0), (-1, 1, 0), (1, 0, -1), (-1, 0, 1), (0, 1, -1), (0, -1, 1)],
}
_W_BY_SPEED = {9: {0: 4 / 9, 1: 1 / 9, 2: 1 / 36}, 19: {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}}


def velocity_set(q: int):
    c = np.array(ORDER[q], dtype=np.int64)
    w = np.array([_W_BY_SPEED[q][int((ci * ci).sum())] for ci in c], dtype=np.float64)
    return c, w


def equilibrium(q: int, rho: np.ndarray, v: np.ndarray) -> np.ndarray:
    """f^eq[i, ...] for rho[...] and v[3, ...] (second-order Maxwellian)."""
    c, w = velocity_set(q)
    cv = np.einsum("ia,a...->i...", c.astype(np.float64), v)
    vv = (v * v).sum(axis=0)
    return w.reshape((-1,) + (1,) * rho.ndim) * rho * (
        1.0 + cv / CS2 + 0.5 * cv * cv / CS2**2 - 0.5 * vv / CS2)


def init(q: int, rho_A: np.ndarray, rho_B: np.ndarray, u=None) -> np.ndarray:
    v = np.zeros((3,) + rho_A.shape) if u is None else np.asarray(u, dtype=np.float64)
    return np.stack([equilibrium(q, rho_A, v), equilibrium(q, rho_B, v)])


def _shift(a: np.ndarray, c) -> np.ndarray:
    """b(x) = a(x + c) on the periodic lattice; arrays are [..., z, y, x]."""
    return np.roll(a, shift=(-int(c[2]), -int(c[1]), -int(c[0])), axis=(-3, -2, -1))


def _opposite(c: np.ndarray) -> np.ndarray:
    """Index of the opposite velocity, found by matching -c_i (vectorised)."""
    match = (c[:, None, :] == -c[None, :, :]).all(axis=2)
    return match.argmax(axis=1)


def _relax(fs, fe, tp, tm, op):
    """BGK when tp == tm, else even / odd parts relaxed with tp / tm."""
    if tp == tm:
        return fs - (fs - fe) / tp
    fp, fm = 0.5 * (fs + fs[op]), 0.5 * (fs - fs[op])
    ep, em = 0.5 * (fe + fe[op]), 0.5 * (fe - fe[op])
    return fs - (fp - ep) / tp - (fm - em) / tm


def step(f: np.ndarray, tau_A: float, tau_B: float, G: float, body_A: float = 0.0,
         forcing: str = "shift", tau_minus=None):
    q = f.shape[1]
    c, w = velocity_set(q)
    cf = c.astype(np.float64)
    rho = f.sum(axis=1)                                   # [s, z, y, x]
    j = np.einsum("sizyx,ia->sazyx", f, cf)               # [s, a, z, y, x]
    # gather of the other species: g_s(x) = sum_i w_i rho_s'(x + c_i) c_i
    gath = np.zeros_like(j)
    for i in range(q):
        for s in range(2):
            nb = _shift(rho[1 - s], c[i])
            gath[s] += w[i] * nb[None] * cf[i].reshape(3, 1, 1, 1)
    F = -G * rho[:, None] * gath
    if body_A != 0.0:
        ny = f.shape[-2]
        y = np.arange(ny, dtype=np.float64).reshape(1, ny, 1)
        F[:, 0] += rho * body_A * np.sin(2.0 * np.pi * y / ny)
    tau = np.array([tau_A, tau_B])
    tm = tau.copy() if tau_minus is None else np.array(
        [tm_ if tm_ > 0 else t_ for tm_, t_ in zip(tau_minus, tau)], dtype=np.float64)
    op = _opposite(c)
    out = np.empty_like(f)
    if forcing == "guo":
        # equilibrium at the common velocity of the half-force corrected momenta,
        # plus each species' discrete forcing term (Hermite projection of F_s),
        # its odd part (c.F) scaled with the odd relaxation time
        u = ((j + 0.5 * F) / tm[:, None, None, None, None]).sum(0) / \
            (rho / tm[:, None, None, None]).sum(0)
        cu = np.einsum("ia,azyx->izyx", cf, u)
        ww = w.reshape(-1, 1, 1, 1)
        for s in range(2):
            cF = np.einsum("ia,azyx->izyx", cf, F[s])
            uF = (u * F[s]).sum(0)
            even = ww * (cu * cF / CS2**2 - uF[None] / CS2)
            odd = ww * cF / CS2
            fs = _relax(f[s], equilibrium(q, rho[s], u), tau[s], tm[s], op)
            fs = fs + (1 - 0.5 / tau[s]) * even + (1 - 0.5 / tm[s]) * odd
            for i in range(q):
                out[s, i] = np.roll(fs[i], shift=(int(c[i, 2]), int(c[i, 1]), int(c[i, 0])),
                                    axis=(-3, -2, -1))
        return out
    u = (j / tm[:, None, None, None, None]).sum(0) / (rho / tm[:, None, None, None]).sum(0)
    for s in range(2):
        v = u + tm[s] * F[s] / rho[s]
        fe = equilibrium(q, rho[s], v)
        fs = _relax(f[s], fe, tau[s], tm[s], op)
        for i in range(q):
            out[s, i] = np.roll(fs[i], shift=(int(c[i, 2]), int(c[i, 1]), int(c[i, 0])),
                                axis=(-3, -2, -1))
    return out


def run(f: np.ndarray, tau_A: float, tau_B: float, G: float, steps: int,
        body_A: float = 0.0, forcing: str = "shift", tau_minus=None) -> np.ndarray:
    g = np.array(f, dtype=np.float64, copy=True)
    for _ in range(steps):
        g = step(g, tau_A, tau_B, G, body_A, forcing, tau_minus)
    return g
