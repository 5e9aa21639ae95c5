"""Pins of the oracle's time step (Sec. 2.1, eq:be and eq. FORCE).

Each test checks the oracle against something other than itself: an exact
permutation, a closed-form discrete sum, a conservation law the method
implies, an independent NumPy implementation, or a Fourier-space
linearisation derived separately (tests/lin_theory.py), which is in turn
checked against the paper's continuum growth rate.
"""
import numpy as np
import pytest

import lin_theory as lt
import oracle
from oracle import twin
import sc_inputs

CS2 = 1.0 / 3.0


# -- streaming ---------------------------------------------------------------

@pytest.mark.parametrize("q,shape", [(9, (1, 5, 7)), (19, (4, 3, 5))])
def test_streaming_is_a_permutation(q, shape):
    c, _ = oracle.lattice(q)
    f = np.zeros((2, q) + shape)
    rng = np.random.default_rng(0)
    f[...] = rng.random(f.shape)
    g = oracle.stream(f)
    # every population moves by exactly c_i (push): g_i(x + c_i) = f_i(x)
    for i in range(q):
        shifted = np.roll(f[:, i], shift=(c[i, 2], c[i, 1], c[i, 0]), axis=(-3, -2, -1))
        assert np.array_equal(g[:, i], shifted)
    assert np.array_equal(np.sort(g.ravel()), np.sort(f.ravel()))


@pytest.mark.parametrize("q,L", [(9, 6), (19, 5)])
def test_lone_population_returns_after_L_steps(q, L):
    c, _ = oracle.lattice(q)
    shape = (L, L, L) if q == 19 else (1, L, L)
    for i in range(1, q):
        f = np.zeros((2, q) + shape)
        f[1, i, 0, 1, 2] = 1.0
        g = f
        for t in range(L):
            g = oracle.stream(g)
            if t < L - 1:
                assert g[1, i, 0, 1, 2] == 0.0   # (t+1) c_i is not 0 mod L yet
        assert np.array_equal(g, f)


# -- force gather --------------------------------------------------------------

@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_force_gather_sine_mode_closed_form(q, axis):
    """psi_B = sin(k x_a): sum_i w_i psi_B(x + c_i) c_i = c_S^2 sin(k) cos(k x_a) e_a.

    The sum over the two velocity classes with c_a = +-1 (total weight 1/6 each)
    gives (1/6)[sin(kx + k) - sin(kx - k)] = (1/3) sin(k) cos(kx) exactly.
    """
    if q == 9 and axis == 2:
        pytest.skip("2D lattice")
    L, m, G = 16, 3, 1.7
    shape = (L, L, L) if q == 19 else (1, L, L)
    k = 2 * np.pi * m / L
    coords = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")  # z, y, x
    xa = coords[2 - axis].astype(float)
    rho = np.stack([np.ones(shape), np.sin(k * xa)])
    F = oracle.force(q, G, rho)
    expect = -G * CS2 * np.sin(k) * np.cos(k * xa)   # F_A = -G psi_A * gather, psi_A = 1
    np.testing.assert_allclose(F[0, axis], expect, rtol=0, atol=1e-14)
    for b in range(3):
        if b != axis:
            np.testing.assert_allclose(F[0, b], 0.0, atol=1e-15)


@pytest.mark.parametrize("q,shape", [(9, (1, 9, 11)), (19, (5, 6, 7))])
def test_force_invariants(q, shape):
    rng = np.random.default_rng(3)
    G = 1.3
    # uniform densities: no force
    F0 = oracle.force(q, G, np.stack([np.full(shape, 0.7), np.full(shape, 0.4)]))
    assert np.abs(F0).max() == 0.0
    # total force sums to zero on any periodic lattice (substitute x -> x - c_i,
    # then pair c_i with -c_i): sum_x (F_A + F_B) = 0
    rho = rng.uniform(0.1, 1.0, (2,) + shape)
    F = oracle.force(q, G, rho)
    tot = (F[0] + F[1]).sum(axis=(1, 2, 3))
    np.testing.assert_allclose(tot, 0.0, atol=1e-12)
    # swapping species swaps the forces
    F2 = oracle.force(q, G, rho[::-1].copy())
    np.testing.assert_array_equal(F2[0], F[1])
    # linear in G
    np.testing.assert_allclose(oracle.force(q, 2 * G, rho), 2 * F, rtol=1e-15, atol=1e-16)


@pytest.mark.parametrize("q", [9, 19])
def test_total_force_is_minus_gradient_of_bulk_pressure(q):
    """Long waves: F_A + F_B -> -grad(c_S^2 G rho_A rho_B), the interaction part of
    the bulk pressure p = c_S^2 (rho_A + rho_B) + c_S^2 G rho_A rho_B (Sec. 2.1)."""
    L, G = 256, 1.3
    shape = (1, 1, L)
    x = np.arange(L, dtype=float).reshape(shape)
    k = 2 * np.pi / L
    rA = 0.6 + 0.05 * np.sin(k * x)
    rB = 0.3 + 0.04 * np.cos(2 * k * x)
    F = oracle.force(q, G, np.stack([rA, rB]))
    dA = 0.05 * k * np.cos(k * x)
    dB = -0.04 * 2 * k * np.sin(2 * k * x)
    expect = -CS2 * G * (rA * dB + rB * dA)
    err = np.abs(F[0, 0] + F[1, 0] - expect).max() / np.abs(expect).max()
    assert err < 2e-3          # O(k^2) lattice correction
    # a wrong prefactor (G/2 or 2G in the pressure) would be off by 50-100 %


# -- conservation and fixed points ------------------------------------------

def test_mass_and_momentum_conservation_cfg1_drop():
    """64x64 D2Q9 drop, tau = 1, G = 1.3: per-species mass conserved to roundoff
    over 2000 steps and total lattice momentum stays at its initial 0.

    Each step can move the total by about one rounding unit of it (sums of
    rounded equilibria are not biased-free), so the bound is steps * 2^-52."""
    fl = sc_inputs.drop(64, 64, 1, radius=16, seed=1)
    f = oracle.init(9, fl.rho_A, fl.rho_B)
    _, _, _, T0 = oracle.observables(f, 1.0, 1.0, 1.3)
    g = oracle.run(f, 1.0, 1.0, 1.3, 2000)
    _, _, _, T = oracle.observables(g, 1.0, 1.0, 1.3)
    for s in ("mass_A", "mass_B"):
        assert abs(T[s] - T0[s]) / T0[s] < 2000 * 2.0**-52
    for a in ("mom_x", "mom_y", "mom_z"):
        assert abs(T[a]) < 1e-12
    assert T["max_u"] > 1e-5          # the drop did evolve (spurious currents)


@pytest.mark.parametrize("q,shape", [(9, (1, 6, 5)), (19, (3, 4, 5))])
def test_uniform_states_are_fixed_points(q, shape):
    rA, rB = np.full(shape, 0.8), np.full(shape, 0.3)
    f = oracle.init(q, rA, rB)
    g = oracle.run(f, 0.7, 1.3, 1.5, 10)
    np.testing.assert_allclose(g, f, rtol=0, atol=1e-15)
    # a uniformly moving state (both species at the same velocity, tau_A = tau_B)
    u = np.zeros((3,) + shape)
    u[0], u[1] = 0.03, -0.02
    if q == 19:
        u[2] = 0.01
    f = oracle.init(q, rA, rB, u)
    g = oracle.run(f, 0.9, 0.9, 1.5, 10)
    np.testing.assert_allclose(g, f, rtol=0, atol=1e-14)


# -- independent implementations ---------------------------------------------

@pytest.mark.parametrize("q,shape", [(9, (1, 8, 8)), (9, (1, 5, 3)), (19, (6, 6, 6)),
                                     (19, (3, 5, 4))])
def test_c_oracle_equals_numpy_twin(q, shape):
    rng = np.random.default_rng(11)
    rA = rng.uniform(0.2, 1.0, shape)
    rB = rng.uniform(0.2, 1.0, shape)
    u = 0.02 * rng.standard_normal((3,) + shape)
    if q == 9:
        u[2] = 0.0
    f = oracle.init(q, rA, rB, u)
    np.testing.assert_array_equal(f, twin.init(q, rA, rB, u))
    a = oracle.run(f, 0.8, 1.1, 1.4, 50, body_A=1e-3)
    b = twin.run(f, 0.8, 1.1, 1.4, 50, body_A=1e-3)
    assert np.abs(a - b).max() <= 1e-14


def test_step_sites_equals_full_step():
    for q, shape in ((9, (1, 7, 9)), (19, (4, 5, 6))):
        rng = np.random.default_rng(5)
        f = oracle.init(q, rng.uniform(0.2, 1, shape), rng.uniform(0.2, 1, shape))
        f = oracle.run(f, 1.0, 0.8, 1.3, 3)
        full = oracle.run(f, 1.0, 0.8, 1.3, 1, body_A=2e-3)
        n = int(np.prod(shape))
        sites = np.array([0, 1, n // 2, n - 1, 17 % n])
        got = oracle.step_sites(f, 1.0, 0.8, 1.3, sites, body_A=2e-3)
        want = full.reshape(2, q, n)[:, :, sites].transpose(2, 0, 1)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)


# -- linearised dynamics -------------------------------------------------------

@pytest.mark.parametrize("q,shape,kvec,n", [
    (9, (1, 32, 32), (2, 1, 0), 15),
    (19, (8, 8, 8), (1, 2, 1), 5),
    (19, (12, 6, 4), (0, 1, 1), 8),
])
def test_oracle_follows_linearised_update(q, shape, kvec, n):
    """A small Fourier-mode perturbation evolves as M(k)^n (independent derivation)."""
    nz, ny, nx = shape
    k = 2 * np.pi * np.array([kvec[0] / nx, kvec[1] / ny, kvec[2] / nz])
    rA0, rB0, tA, tB, G = 0.6, 0.4, 0.9, 1.2, 1.5
    M = lt.update_matrix(q, k, rA0, rB0, tA, tB, G)
    rng = np.random.default_rng(1)
    vh = rng.standard_normal(2 * q) + 1j * rng.standard_normal(2 * q)
    c, w = lt.vset(q)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ph = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z))
    f0 = np.stack([rA0 * w, rB0 * w])[:, :, None, None, None]
    eps = 1e-7

    def field(v):
        return f0 + eps * np.real(v.reshape(2, q)[:, :, None, None, None] * ph)

    got = oracle.run(field(vh), tA, tB, G, n)
    want = field(np.linalg.matrix_power(M, n) @ vh)
    signal = np.abs(want - f0).max()
    assert signal > 1e-8
    assert np.abs(got - want).max() < 1e-5 * signal


@pytest.mark.parametrize("rho,tau,G", [(1.0, 1.0, 0.5), (1.4, 0.55, 0.164), (1.0, 0.7, 1.0),
                                       (1.05, 1.0, 1.3)])
def test_linear_phi_rate_matches_paper_continuum_limit(rho, tau, G):
    """The order-parameter eigenvalue of M(k) reproduces, as k -> 0, the growth
    rate of the paper's linearised chemical potential with g^(tau) = tau G/(tau - 1/2):
    omega/k^2 -> -(tau - 1/2) c_S^2 + rho tau G c_S^2 / 2 (Sec. 2.1)."""
    a = -(tau - 0.5) * CS2 + rho * tau * G * CS2 / 2
    for q, kdir in ((9, (1, 0, 0)), (9, (0.6, 0.8, 0)), (19, (0, 0, 1))):
        r = []
        for kk in (0.01, 0.02):
            kv = kk * np.array(kdir)
            r.append(lt.phi_mode_rate(q, kv, rho, tau, G).real / kk**2)
        # Richardson extrapolation of the O(k^2) correction to k = 0
        lim = (4 * r[0] - r[1]) / 3
        assert abs(lim - a) < 1e-6 * max(abs(a), 1e-3)
    # the paper's full O(k^4) expression is close at small k, too
    kk = 0.02
    assert abs(lt.phi_mode_rate(9, (kk, 0, 0), rho, tau, G).real
               - lt.paper_phi_rate(kk, rho, tau, G)) < 0.01 * abs(a) * kk**2


@pytest.mark.parametrize("q,shape,forcing,tm", [(9, (1, 40, 36), "shift", None),
                                                (19, (10, 12, 14), "guo", None),
                                                (19, (9, 8, 7), "shift", (0.8, 1.3))])
def test_all_core_build_equals_single_thread(q, shape, forcing, tm):
    """The OpenMP build of the oracle (used to time it on all host cores) runs
    the same per-site arithmetic: its populations equal the default build's."""
    fl = sc_inputs.drop(shape[2], shape[1], shape[0], radius=min(shape[1:]) / 4, seed=9)
    f0 = oracle.init(q, fl.rho_A, fl.rho_B)
    a = oracle.run(f0, 0.9, 1.1, 1.4, 12, body_A=1e-5, forcing=forcing, tau_minus=tm)
    b = oracle.run(f0, 0.9, 1.1, 1.4, 12, body_A=1e-5, forcing=forcing, tau_minus=tm,
                   all_cores=True)
    assert np.array_equal(a, b)
