"""Pins of the oracle's two-relaxation-time collision (tau_minus): the even
part of each species' deviation from equilibrium relaxes with tau_s = tau+,
the odd part with tau- -- the member of the multiple-relaxation-time family
that decouples the viscous and diffusive time scales, which the paper names
as the way to do so (Sec. 2.1, closing remark).

* the C oracle equals the independently written NumPy twin (both forcings);
* tau- = tau+ is the BGK step bit for bit;
* shear waves decay with nu = c_S^2 (tau+ - 1/2) and order-parameter waves
  with D = c_S^2 (tau- - 1/2), independently of each other;
* small Fourier modes follow the separately derived linearised update;
* the order-parameter growth rate tends to the continuum limit with mobility
  c_S^2 (tau- - 1/2) and coupling tau- g / (tau- - 1/2) (velocity shift) or g
  (Guo forcing): tau+ drops out of the diffusion;
* Guo with two relaxation times still conserves mass and adds sum_s F_s.
"""
import numpy as np
import pytest

import lin_theory as lt
import oracle
from oracle import twin

CS2 = 1.0 / 3.0


@pytest.mark.parametrize("forcing", ["shift", "guo"])
@pytest.mark.parametrize("q,shape", [(9, (1, 8, 8)), (19, (5, 6, 4))])
def test_c_oracle_equals_numpy_twin_with_two_relaxation_times(q, shape, forcing):
    rng = np.random.default_rng(11)
    rA, rB = rng.uniform(0.3, 1.0, shape), rng.uniform(0.3, 1.0, shape)
    f = oracle.init(q, rA, rB)
    tm = (1.3, 0.7)
    a = oracle.run(f, 0.8, 1.1, 1.4, 40, body_A=1e-3, forcing=forcing, tau_minus=tm)
    b = twin.run(f, 0.8, 1.1, 1.4, 40, body_A=1e-3, forcing=forcing, tau_minus=tm)
    assert np.abs(a - b).max() < 1e-13


def test_equal_relaxation_times_are_the_bgk_step():
    rng = np.random.default_rng(2)
    shape = (1, 9, 11)
    f = oracle.init(9, rng.uniform(0.3, 1, shape), rng.uniform(0.3, 1, shape))
    for forcing in ("shift", "guo"):
        a = oracle.run(f, 0.9, 1.2, 1.3, 20, forcing=forcing)
        b = oracle.run(f, 0.9, 1.2, 1.3, 20, forcing=forcing, tau_minus=(0.9, 1.2))
        assert np.array_equal(a, b)


def _wave_rate(q, tp, tm, kind):
    L = 64
    k = 2 * np.pi / L
    if kind == "shear":
        shape = (1, L, 1)
        y = np.arange(L, dtype=float).reshape(1, L, 1)
        u = np.zeros((3,) + shape)
        u[0] = 1e-4 * np.sin(k * y)
        f = oracle.init(q, np.full(shape, 0.5), np.full(shape, 0.5), u)
        probe, coord = (lambda g: oracle.observables(g, tp, tp, 0.0)[1][0]), y
        n1, n2 = 100, 700
    else:
        shape = (1, 1, L)
        x = np.arange(L, dtype=float).reshape(1, 1, L)
        phi = 1e-4 * np.sin(k * x)
        f = oracle.init(q, 0.5 + phi / 2, 0.5 - phi / 2)

        def probe(g):
            r = g.sum(axis=1)
            return r[0] - r[1]
        coord, n1, n2 = x, 100, 900
    g1 = oracle.run(f, tp, tp, 0.0, n1, tau_minus=(tm, tm))
    g2 = oracle.run(g1, tp, tp, 0.0, n2 - n1, tau_minus=(tm, tm))
    a1 = 2 * np.mean(probe(g1) * np.sin(k * coord))
    a2 = 2 * np.mean(probe(g2) * np.sin(k * coord))
    return -np.log(a2 / a1) / ((n2 - n1) * k * k)


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("tp,tm", [(0.8, 1.4), (1.2, 0.6)])
def test_viscosity_follows_tau_plus_and_diffusion_tau_minus(q, tp, tm):
    nu = _wave_rate(q, tp, tm, "shear")
    D = _wave_rate(q, tp, tm, "phi")
    assert abs(nu - CS2 * (tp - 0.5)) < 5e-3 * CS2 * (tp - 0.5)
    assert abs(D - CS2 * (tm - 0.5)) < 5e-3 * CS2 * (tm - 0.5)


@pytest.mark.parametrize("forcing", ["shift", "guo"])
def test_oracle_follows_linearised_two_relaxation_time_update(forcing):
    q, shape, kvec, n = 9, (1, 32, 32), (2, 1, 0), 15
    nz, ny, nx = shape
    k = 2 * np.pi * np.array([kvec[0] / nx, kvec[1] / ny, kvec[2] / nz])
    rA0, rB0, tA, tB, G, tm = 0.6, 0.4, 0.9, 1.2, 1.5, (0.7, 1.4)
    M = lt.update_matrix(q, k, rA0, rB0, tA, tB, G, forcing, tm)
    rng = np.random.default_rng(1)
    vh = rng.standard_normal(2 * q) + 1j * rng.standard_normal(2 * q)
    c, w = lt.vset(q)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ph = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z))
    f0 = np.stack([rA0 * w, rB0 * w])[:, :, None, None, None]
    eps = 1e-7

    def field(v):
        return f0 + eps * np.real(v.reshape(2, q)[:, :, None, None, None] * ph)

    got = oracle.run(field(vh), tA, tB, G, n, forcing=forcing, tau_minus=tm)
    want = field(np.linalg.matrix_power(M, n) @ vh)
    signal = np.abs(want - f0).max()
    assert np.abs(got - want).max() < 1e-5 * signal


@pytest.mark.parametrize("forcing", ["shift", "guo"])
@pytest.mark.parametrize("rho,tp,tm,G", [(1.0, 0.8, 0.6, 0.5), (1.0, 1.2, 0.7, 0.8),
                                         (1.0, 0.6, 1.1, 1.0)])
def test_growth_rate_has_the_odd_relaxation_time_only(rho, tp, tm, G, forcing):
    g = tm * G / (tm - 0.5) if forcing == "shift" else G
    a = -(tm - 0.5) * CS2 * (1 - rho * g / 2)
    r = [lt.phi_mode_rate(9, (kk, 0, 0), rho, tp, G, forcing, tm).real / kk**2
         for kk in (0.01, 0.02)]
    lim = (4 * r[0] - r[1]) / 3
    assert abs(lim - a) < 1e-6 * max(abs(a), 1e-3)


def test_guo_with_two_relaxation_times_balances_mass_and_momentum():
    rng = np.random.default_rng(4)
    q, shape, tA, tB, G, A = 19, (4, 5, 6), 0.7, 1.1, 1.5, 2e-3
    tm = (1.4, 0.6)
    f = oracle.init(q, rng.uniform(0.3, 1.0, shape), rng.uniform(0.3, 1.0, shape))
    f = oracle.run(f, tA, tB, G, 3, forcing="guo", tau_minus=tm)
    post = oracle.collide(f, tA, tB, G, body_A=A, forcing="guo", tau_minus=tm)
    c, _ = lt.vset(q)
    rho = f.sum(axis=1)
    np.testing.assert_allclose(post.sum(axis=1), rho, rtol=1e-14, atol=0)
    F = oracle.force(q, G, rho)
    ny = shape[1]
    y = np.arange(ny, dtype=float).reshape(1, ny, 1)
    F[:, 0] += rho * A * np.sin(2 * np.pi * y / ny)
    j_pre = np.einsum("sizyx,ia->azyx", f, c)
    j_post = np.einsum("sizyx,ia->azyx", post, c)
    assert np.abs(j_post - (j_pre + F.sum(axis=0))).max() < 1e-14
