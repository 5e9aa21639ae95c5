"""Pins of the oracle's reduced observables that the GPU totals are checked
against: the total kinetic energy and the droplet node count of Sec. 4.2.

* The kinetic energy is the integral of u_x^2 + u_y^2 over the domain (the
  quantity plotted in the paper's Fig. 6): on the lattice, the plain sum of
  |u_phys|^2 over the sites, not weighted by density and without a factor 1/2.
  Pinned by two closed forms: a state in uniform motion (no force acts, so
  u_phys is the imposed velocity everywhere) and the laminar Kolmogorov flow
  of Sec. 4.2 at G = 0, u_x = A / (nu k^2) sin(k y), whose sum over a period
  is N (A / (nu k^2))^2 / 2.
* The droplet node count M(t) of the leakage L(t) = M(t) / M_0 counts sites
  with phi = rho_A - rho_B >= phi_T, phi_T = 0 (Sec. 4.2): pinned on a field
  with a hand-made sign pattern that includes sites where phi is exactly 0.
"""
import numpy as np
import pytest

import oracle

CS2 = 1.0 / 3.0


@pytest.mark.parametrize("q,shape", [(9, (1, 7, 5)), (19, (4, 5, 6))])
def test_kinetic_energy_of_uniform_motion(q, shape):
    """f = f^eq(rho_s, u0) everywhere: no force, u_phys = u0, ke = N |u0|^2."""
    u0 = np.array([0.01, -0.02, 0.005 if q == 19 else 0.0])
    u = np.broadcast_to(u0.reshape(3, 1, 1, 1), (3,) + shape).copy()
    f = oracle.init(q, np.full(shape, 0.3), np.full(shape, 0.9), u)
    _, uu, _, T = oracle.observables(f, 1.0, 1.0, 1.3)
    n = int(np.prod(shape))
    expect = n * float(u0 @ u0)
    assert abs(T["ke"] - expect) <= 1e-12 * expect
    assert abs(T["max_u"] - np.sqrt(u0 @ u0)) <= 1e-12
    # ke is a plain sum: independent of the density (rho = 1.2 here)
    assert np.allclose(uu.reshape(3, -1).T, u0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("nx", [1, 6])
def test_kinetic_energy_of_laminar_kolmogorov_flow(nx):
    """G = 0, rho = 1.4: F_x = rho A sin(2 pi y / L) drives u_x = U sin(ky) with
    U = A / (nu k^2); the total kinetic energy is N U^2 / 2 and max |u| = U."""
    L, tau, A = 32, 1.0, 1e-6
    shape = (1, L, nx)
    f = oracle.init(9, np.full(shape, 0.7), np.full(shape, 0.7))
    f = oracle.run(f, tau, tau, 0.0, 3000, body_A=A)
    _, _, _, T = oracle.observables(f, tau, tau, 0.0, body_A=A)
    k = 2 * np.pi / L
    U = A / (CS2 * (tau - 0.5) * k * k)
    n = L * nx
    assert abs(T["ke"] - n * U * U / 2) <= 1e-2 * n * U * U / 2
    assert abs(T["max_u"] - U) <= 1e-2 * U


@pytest.mark.parametrize("q,shape", [(9, (1, 6, 8)), (19, (3, 4, 5))])
def test_droplet_node_count_sign_pattern(q, shape):
    """n_phi_pos counts phi >= 0: positive sites and sites with phi exactly 0."""
    rng = np.random.default_rng(11)
    n = int(np.prod(shape))
    sign = rng.integers(-1, 2, size=n)          # -1, 0, +1 per site
    d = 0.05 * sign * rng.uniform(0.2, 1.0, size=n)
    d[sign == 0] = 0.0
    rho_A = (0.6 + d).reshape(shape)
    rho_B = (0.6 - d).reshape(shape)
    f = oracle.init(q, rho_A, rho_B)
    rho, _, _, T = oracle.observables(f, 1.0, 1.0, 1.3)
    phi = (rho[0] - rho[1]).ravel()
    # equal densities give bitwise equal populations, so phi is exactly 0 there
    assert np.all(phi[sign == 0] == 0.0)
    assert np.all(np.sign(phi) == sign)
    expect = int(np.sum(sign > 0) + np.sum(sign == 0))
    assert 0 < np.sum(sign == 0) < n and np.sum(sign > 0) > 0
    assert T["n_phi_pos"] == expect
