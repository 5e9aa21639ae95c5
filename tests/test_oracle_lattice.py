"""Pins of the oracle's velocity sets and equilibrium (Sec. 2.1).

The paper fixes the weights only through their normalisation (second- and
fourth-order isotropy with c_S^2 = 1/3) and the equilibrium only as a local
Maxwellian truncated at second order; these tests check both properties
exactly (rational arithmetic) or to roundoff.
"""
from fractions import Fraction
import itertools

import numpy as np
import pytest

import oracle
from oracle import twin


def _frac_weights(w):
    fr = [Fraction(x).limit_denominator(1000) for x in w]
    for x, f in zip(w, fr):
        assert abs(float(f) - x) <= 2e-16 * max(1.0, abs(x))
    return fr


@pytest.mark.parametrize("q", [9, 19])
def test_isotropy_sums_exact(q):
    c, w = oracle.lattice(q)
    W = _frac_weights(w)
    D = 2 if q == 9 else 3
    cs2 = Fraction(1, 3)
    assert sum(W) == 1
    assert len({tuple(ci) for ci in c}) == q          # distinct velocities
    for a in range(3):
        assert sum(Wi * int(ci[a]) for Wi, ci in zip(W, c)) == 0
    for a, b in itertools.product(range(D), repeat=2):
        s = sum(Wi * int(ci[a]) * int(ci[b]) for Wi, ci in zip(W, c))
        assert s == (cs2 if a == b else 0)
    # third moments vanish (odd)
    for a, b, g in itertools.product(range(D), repeat=3):
        assert sum(Wi * int(ci[a] * ci[b] * ci[g]) for Wi, ci in zip(W, c)) == 0
    # fourth-order isotropy: c_S^4 (d_ab d_gk + d_ag d_bk + d_ak d_bg)
    d = lambda i, j: 1 if i == j else 0
    for a, b, g, k in itertools.product(range(D), repeat=4):
        s = sum(Wi * int(ci[a] * ci[b] * ci[g] * ci[k]) for Wi, ci in zip(W, c))
        assert s == cs2 * cs2 * (d(a, b) * d(g, k) + d(a, g) * d(b, k) + d(a, k) * d(b, g))
    # one-sided sum used by the closed-form gather: sum_{c_x = +1} w = 1/6
    assert sum(Wi for Wi, ci in zip(W, c) if ci[0] == 1) == Fraction(1, 6)
    if q == 9:
        assert all(ci[2] == 0 for ci in c)


@pytest.mark.parametrize("q", [9, 19])
def test_oracle_tables_match_speed_class_rule(q):
    c, w = oracle.lattice(q)
    c2, w2 = twin.velocity_set(q)
    assert np.array_equal(c, c2)
    assert np.array_equal(w, w2)


@pytest.mark.parametrize("q", [9, 19])
def test_equilibrium_moments(q):
    c, _ = oracle.lattice(q)
    cf = c.astype(float)
    rng = np.random.default_rng(7)
    D = 2 if q == 9 else 3
    for _ in range(20):
        rho = rng.uniform(0.01, 2.0)
        v = np.zeros(3)
        v[:D] = rng.uniform(-0.2, 0.2, D)
        fe = oracle.feq(q, rho, v)
        assert abs(fe.sum() - rho) <= 1e-15 * 4
        np.testing.assert_allclose(fe @ cf, rho * v, rtol=0, atol=2e-15)
        Pi = np.einsum("i,ia,ib->ab", fe, cf, cf)
        expect = rho * (np.eye(3) / 3.0 + np.outer(v, v))
        if q == 9:
            expect[2, 2] = 0.0   # no z motion on a 2D lattice
        np.testing.assert_allclose(Pi, expect, rtol=0, atol=4e-15)


def test_zero_velocity_equilibrium_is_weights():
    for q in (9, 19):
        _, w = oracle.lattice(q)
        np.testing.assert_array_equal(oracle.feq(q, 1.0, [0, 0, 0]), w)
