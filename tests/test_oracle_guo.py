"""Pins of the oracle's Guo forcing option (the discrete forcing the paper
cites, Sec. 2.3, as the cure for the tau-dependent coupling g^(tau)).

* the C oracle equals the independently written NumPy twin (brute force on
  small grids, unequal tau_A / tau_B, with the Kolmogorov body force);
* exact balances of one collision: each species' mass is unchanged and the
  total momentum grows by exactly sum_s F_s (any tau_s);
* the linearised update M(k) of the scheme (derived separately) predicts a
  small Fourier mode's evolution;
* the order-parameter growth rate tends, as k -> 0, to the paper's continuum
  limit with the bare coupling G in place of g^(tau) = tau G / (tau - 1/2):
  the tau-dependence the paper attributes to the velocity shift is gone, and
  the same parameters that phase-separate under the shift are stable here;
* G = 0 Kolmogorov forcing reaches the laminar profile A / (nu k^2) sin(k y).
"""
import numpy as np
import pytest

import lin_theory as lt
import oracle
from oracle import twin

CS2 = 1.0 / 3.0


@pytest.mark.parametrize("q,shape", [(9, (1, 8, 8)), (19, (6, 6, 6)), (19, (4, 5, 7))])
def test_c_oracle_equals_numpy_twin_with_guo_forcing(q, shape):
    rng = np.random.default_rng(7)
    rA, rB = rng.uniform(0.3, 1.0, shape), rng.uniform(0.3, 1.0, shape)
    u = rng.uniform(-0.02, 0.02, (3,) + shape)
    if q == 9:
        u[2] = 0.0
    f = oracle.init(q, rA, rB, u)
    a = oracle.run(f, 0.8, 1.1, 1.4, 50, body_A=1e-3, forcing="guo")
    b = twin.run(f, 0.8, 1.1, 1.4, 50, body_A=1e-3, forcing="guo")
    assert np.abs(a - b).max() < 1e-13


@pytest.mark.parametrize("q,shape,tA,tB", [(9, (1, 9, 7), 0.7, 1.3), (19, (5, 4, 6), 1.0, 1.0),
                                          (19, (4, 6, 5), 0.55, 0.9)])
def test_one_collision_conserves_mass_and_adds_the_force(q, shape, tA, tB):
    rng = np.random.default_rng(3)
    f = oracle.init(q, rng.uniform(0.3, 1.0, shape), rng.uniform(0.3, 1.0, shape))
    f = oracle.run(f, tA, tB, 1.5, 3, forcing="guo")
    G, A = 1.5, 2e-3
    post = oracle.collide(f, tA, tB, G, body_A=A, forcing="guo")
    c, _ = lt.vset(q)
    rho = f.sum(axis=1)
    np.testing.assert_allclose(post.sum(axis=1), rho, rtol=1e-14, atol=0)
    F = oracle.force(q, G, rho)                          # [s, a, ...]
    ny = shape[1]
    y = np.arange(ny, dtype=float).reshape(1, ny, 1)
    F[:, 0] += rho * A * np.sin(2 * np.pi * y / ny)
    j_pre = np.einsum("sizyx,ia->azyx", f, c)
    j_post = np.einsum("sizyx,ia->azyx", post, c)
    assert np.abs(j_post - (j_pre + F.sum(axis=0))).max() < 1e-14


@pytest.mark.parametrize("q,shape,kvec,n", [(9, (1, 32, 32), (2, 1, 0), 15),
                                            (19, (8, 8, 8), (1, 2, 1), 5)])
def test_oracle_follows_linearised_guo_update(q, shape, kvec, n):
    nz, ny, nx = shape
    k = 2 * np.pi * np.array([kvec[0] / nx, kvec[1] / ny, kvec[2] / nz])
    rA0, rB0, tA, tB, G = 0.6, 0.4, 0.9, 1.2, 1.5
    M = lt.update_matrix(q, k, rA0, rB0, tA, tB, G, forcing="guo")
    rng = np.random.default_rng(1)
    vh = rng.standard_normal(2 * q) + 1j * rng.standard_normal(2 * q)
    c, w = lt.vset(q)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ph = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z))
    f0 = np.stack([rA0 * w, rB0 * w])[:, :, None, None, None]
    eps = 1e-7

    def field(v):
        return f0 + eps * np.real(v.reshape(2, q)[:, :, None, None, None] * ph)

    got = oracle.run(field(vh), tA, tB, G, n, forcing="guo")
    want = field(np.linalg.matrix_power(M, n) @ vh)
    signal = np.abs(want - f0).max()
    assert signal > 1e-8
    assert np.abs(got - want).max() < 1e-5 * signal


@pytest.mark.parametrize("rho,tau,G", [(1.4, 0.55, 0.164), (1.0, 0.7, 1.0), (1.0, 0.55, 0.3),
                                       (1.05, 1.0, 1.3)])
def test_guo_growth_rate_has_the_bare_coupling(rho, tau, G):
    """omega / k^2 -> -(tau - 1/2) c_S^2 (1 - rho G / 2): the paper's limit with
    g^(tau) replaced by G."""
    a = -(tau - 0.5) * CS2 * (1 - rho * G / 2)
    for q, kdir in ((9, (1, 0, 0)), (9, (0.6, 0.8, 0)), (19, (0, 0, 1))):
        r = []
        for kk in (0.01, 0.02):
            r.append(lt.phi_mode_rate(q, kk * np.array(kdir), rho, tau, G, "guo").real / kk**2)
        lim = (4 * r[0] - r[1]) / 3
        assert abs(lim - a) < 1e-6 * max(abs(a), 1e-3)
    kk = 0.02
    assert abs(lt.phi_mode_rate(9, (kk, 0, 0), rho, tau, G, "guo").real
               - lt.paper_phi_rate(kk, rho, tau, G, coupling="g")) < 0.01 * abs(a) * kk**2


def test_same_parameters_separate_under_the_shift_but_not_under_guo():
    """tau = 0.55, rho = 1, G = 0.3: rho g^(tau) = 3.3 > 2 (spinodal under the
    velocity shift) while rho G = 0.3 < 2 (stable under Guo forcing).  A small
    phi sine grows with one scheme and decays with the other in the oracle."""
    L, tau, G, rho = 32, 0.55, 0.3, 1.0
    x = np.arange(L, dtype=float).reshape(1, 1, L)
    phi = 1e-6 * np.sin(2 * np.pi * 4 * x / L)
    f = oracle.init(9, rho / 2 + phi / 2, rho / 2 - phi / 2)
    amp = {}
    for scheme in ("shift", "guo"):
        g = oracle.run(f, tau, tau, G, 400, forcing=scheme)
        r = g.sum(axis=1)
        amp[scheme] = np.abs(r[0] - r[1]).max()
    # linear rates at this k: +4.4e-3 per step (shift), -9.4e-3 (Guo)
    assert amp["shift"] > 3e-6 and amp["guo"] < 1e-7


def test_kolmogorov_profile_with_guo_forcing():
    L, tau, A = 32, 1.0, 1e-6
    shape = (1, L, 1)
    f = oracle.init(9, np.full(shape, 0.5), np.full(shape, 0.5))
    f = oracle.run(f, tau, tau, 0.0, 3000, body_A=A, forcing="guo")
    u = oracle.observables(f, tau, tau, 0.0, body_A=A)[1][0]
    y = np.arange(L, dtype=float).reshape(1, L, 1)
    k = 2 * np.pi / L
    amp = 2.0 * np.mean(u * np.sin(k * y))
    expect = A / (CS2 * (tau - 0.5) * k * k)
    assert abs(amp - expect) / expect < 1e-2
    assert abs(2.0 * np.mean(u * np.cos(k * y))) < 1e-3 * expect
