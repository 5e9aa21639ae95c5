"""Full-size checks in the benchmark's launch configuration.

At 256^3 D3Q19 a full oracle step takes about half a minute, so the step is
checked on sampled sites the oracle computes one by one (oracle.step_sites),
and the run over many steps through properties that hold at any size (mass
per species conserved to roundoff, lattice momentum stays zero).
"""
import numpy as np
import pytest

import oracle
import sc_inputs
from gpu_common import say

pytestmark = pytest.mark.gpu

L = 256
G, TAU = 1.6, 1.0


@pytest.fixture(scope="module")
def spinodal256():
    return sc_inputs.spinodal(L, L, L, seed=3)


def _sample_sites(n, k, seed):
    rng = np.random.default_rng(seed)
    s = rng.integers(0, n, size=k)
    # plus lattice corners and planes at the march-chunk and tile edges
    extra = [0, n - 1, L - 1, L * L - 1, L * L, 63, 64, 31 * L * L + 5 * L + 7,
             32 * L * L + 4 * L + 64]
    return np.unique(np.concatenate([s, extra])).astype(np.int64)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_shifted", 2e-6)])
def test_256cube_one_step_sampled(spinodal256, precision, tol):
    from paper_1112_5547_amd import Lattice
    fl = spinodal256
    say(f"256^3 D3Q19 {precision}: init + 1 step (benchmark kernel config)")
    lat = Lattice(19, L, L, L, tau_A=TAU, G=G, precision=precision)
    lat.init(fl.rho_A, fl.rho_B)
    lat.step(1)
    f = lat.get_populations().reshape(2, 19, -1)
    lat.close()
    f0 = oracle.init(19, fl.rho_A, fl.rho_B)
    sites = _sample_sites(L ** 3, 3000, 1)
    want = oracle.step_sites(f0, TAU, TAU, G, sites)
    got = f[:, :, sites].transpose(2, 0, 1)
    assert float(np.abs(got - want).max()) <= tol


def test_256cube_conservation_over_200_steps(spinodal256):
    from paper_1112_5547_amd import Lattice
    fl = spinodal256
    say("256^3 D3Q19 fp64: 200 steps, mass and momentum")
    lat = Lattice(19, L, L, L, tau_A=TAU, G=G)
    lat.init(fl.rho_A, fl.rho_B)
    T0 = lat.totals()
    lat.step(200)
    T = lat.totals()
    for s in ("mass_A", "mass_B"):
        assert abs(T[s] - T0[s]) <= 200 * 2.0 ** -52 * T0[s] * 4
    for a in ("mom_x", "mom_y", "mom_z"):
        assert abs(T[a]) <= 1e-9
    assert T["n_nonfinite"] == 0
