"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bar: FP64 populations within 1e-12 max-abs of the oracle after the stated
steps (the two sides differ only in rounding order: FMA contraction and the
multiplication by 1/tau instead of a division).  Inputs are the seeded
generators of sc_inputs, identical host arrays on both sides.
"""
import numpy as np
import pytest

import oracle
import sc_inputs
from gpu_common import gpu_run, maxabs, oracle_run, say

pytestmark = pytest.mark.gpu

TOL = 1e-12


def test_cfg1_d2q9_drop_100_steps():
    """64x64 D2Q9 drop R = 16, tau = 1, G = 1.3, noise 1e-3 (seed 1)."""
    fl = sc_inputs.drop(64, 64, 1, radius=16, seed=1)
    say("cfg1 D2Q9 64x64 fp64 fused default tile, 100 steps")
    lat, f = gpu_run(9, fl.rho_A, fl.rho_B, 1.0, 1.0, 1.3, 100)
    ref = oracle_run(9, fl.rho_A, fl.rho_B, 1.0, 1.0, 1.3, 100)
    assert maxabs(f, ref) <= TOL
    assert np.abs(ref - oracle.init(9, fl.rho_A, fl.rho_B)).max() > 1e-3  # it moved


@pytest.mark.parametrize("kernel", [(0, 64, 1, 5), (0, 128, 1, 64), (0, 256, 1, 7),
                                    (0, 512, 1, 3), (1, 64, 1, 8), (2, 64, 1, 5), (2, 128, 1, 1),
                                    (2, 256, 1, 37), (2, 512, 1, 2), (3, 64, 1, 5),
                                    (3, 128, 1, 1), (3, 256, 1, 37), (3, 512, 1, 2)])
def test_d2q9_ragged_tiles_and_variants(kernel):
    """100 x 37 (ragged against every tile), unequal tau, body force."""
    fl = sc_inputs.drop(100, 37, 1, radius=9, seed=11)
    say(f"D2Q9 100x37 kernel={kernel}, 60 steps")
    _, f = gpu_run(9, fl.rho_A, fl.rho_B, 0.8, 1.2, 1.5, 60, kernel=kernel, body_A=1e-4)
    ref = oracle_run(9, fl.rho_A, fl.rho_B, 0.8, 1.2, 1.5, 60, body_A=1e-4)
    assert maxabs(f, ref) <= TOL


def test_d3q19_drop_32cube_100_steps():
    fl = sc_inputs.drop(32, 32, 32, radius=8, seed=2)
    say("D3Q19 32^3 drop fp64 default kernel, 100 steps")
    _, f = gpu_run(19, fl.rho_A, fl.rho_B, 1.0, 1.0, 1.3, 100)
    ref = oracle_run(19, fl.rho_A, fl.rho_B, 1.0, 1.0, 1.3, 100)
    assert maxabs(f, ref) <= TOL


@pytest.mark.parametrize("kernel", [(0, 32, 4, 3), (0, 64, 4, 11), (0, 32, 8, 4), (0, 64, 8, 2),
                                    (0, 16, 16, 5), (0, 32, 16, 11), (1, 32, 4, 8), (2, 32, 4, 3),
                                    (2, 64, 4, 11), (2, 32, 8, 1), (2, 64, 8, 2), (2, 16, 16, 5),
                                    (2, 32, 16, 11), (3, 32, 4, 3), (3, 64, 4, 11), (3, 32, 8, 1),
                                    (3, 64, 8, 2), (3, 16, 16, 5), (3, 32, 16, 11)])
def test_d3q19_ragged_tiles_and_variants(kernel):
    """37 x 29 x 11 spinodal (ragged in x, y and the march), unequal tau."""
    fl = sc_inputs.spinodal(37, 29, 11, seed=12)
    say(f"D3Q19 37x29x11 kernel={kernel}, 40 steps")
    _, f = gpu_run(19, fl.rho_A, fl.rho_B, 0.9, 1.1, 1.6, 40, kernel=kernel, body_A=2e-4)
    ref = oracle_run(19, fl.rho_A, fl.rho_B, 0.9, 1.1, 1.6, 40, body_A=2e-4)
    assert maxabs(f, ref) <= TOL


def test_default_kernel_configuration():
    """A new handle starts with the documented configuration: D3Q19 64 x 8
    tiles (32 x 4 for nx <= 32), fused in FP64, pipelined in FP32 shifted,
    march chunks of about one block per compute unit."""
    from paper_1112_5547_amd import Lattice
    cases = [((19, 128, 128, 128, "fp64"), (0, 64, 8, 16)),
             ((19, 128, 128, 128, "fp32_shifted"), (2, 64, 8, 16)),
             ((19, 32, 32, 32, "fp64"), (0, 32, 4, 8)),
             ((9, 1024, 1024, 1, "fp64"), (0, 256, 1, 8))]
    for (q, nx, ny, nz, prec), expect in cases:
        lat = Lattice(q, nx, ny, nz, tau_A=1.0, G=1.3, precision=prec)
        assert lat.kernel == expect, (q, nx, ny, nz, prec, lat.kernel)
        lat.close()


@pytest.mark.parametrize("q,shape,kernel", [
    (19, (40, 43, 41), (0, 64, 8, 16)), (19, (40, 43, 41), (2, 32, 8, 7)),
    (19, (40, 43, 41), (1, 32, 4, 8)), (9, (1, 251, 263), (2, 256, 1, 9)),
    (9, (1, 251, 263), (3, 128, 1, 5))])
def test_padded_array_stride_ragged(q, shape, kernel):
    """Lattices of more than 2^16 sites whose N is not a multiple of 32: the
    population arrays are N rounded up to 32 plus 2080 elements apart, so
    every array base other than the first is offset from N * (s Q + i)."""
    nz, ny, nx = shape
    assert nx * ny * nz >= 1 << 16 and (nx * ny * nz) % 32 != 0
    if q == 19:
        fl = sc_inputs.spinodal(nx, ny, nz, seed=21)
    else:
        fl = sc_inputs.drop(nx, ny, 1, radius=40, seed=21)
    steps = 12 if q == 19 else 40
    say(f"padded stride q={q} shape={shape} kernel={kernel}, {steps} steps")
    _, f = gpu_run(q, fl.rho_A, fl.rho_B, 0.9, 1.2, 1.5, steps, kernel=kernel, body_A=1e-4)
    ref = oracle_run(q, fl.rho_A, fl.rho_B, 0.9, 1.2, 1.5, steps, body_A=1e-4)
    assert maxabs(f, ref) <= TOL


@pytest.mark.parametrize("q,shape", [(9, (1, 5, 1)), (9, (1, 1, 7)), (9, (1, 2, 3)),
                                     (19, (6, 1, 1)), (19, (1, 4, 5)), (19, (2, 3, 2)),
                                     (19, (1, 1, 1))])
def test_degenerate_shapes(q, shape):
    """Extents of 1 and 2: a site is its own (or its neighbour's) periodic image."""
    rng = np.random.default_rng(sum(shape) + q)
    rA = rng.uniform(0.3, 0.9, shape)
    rB = rng.uniform(0.3, 0.9, shape)
    say(f"degenerate q={q} shape={shape}, 20 steps")
    _, f = gpu_run(q, rA, rB, 0.9, 1.3, 1.4, 20)
    ref = oracle_run(q, rA, rB, 0.9, 1.3, 1.4, 20)
    assert maxabs(f, ref) <= TOL


def test_zero_steps_is_the_initial_equilibrium():
    fl = sc_inputs.drop(20, 16, 1, radius=4, seed=5)
    u = np.zeros((3, 1, 16, 20))
    u[0] = 0.01
    u[1] = -0.02
    say("D2Q9 init with velocity, 0 steps")
    _, f = gpu_run(9, fl.rho_A, fl.rho_B, 1.0, 1.0, 1.3, 0, u=u)
    ref = oracle.init(9, fl.rho_A, fl.rho_B, u)
    assert maxabs(f, ref) <= 1e-15


def test_observables_match_oracle():
    fl = sc_inputs.drop(64, 64, 1, radius=16, seed=1)
    say("cfg1 observables after 100 steps")
    lat, f = gpu_run(9, fl.rho_A, fl.rho_B, 1.0, 1.0, 1.3, 100)
    lat.set_probe(*fl.centre, 16.0)
    rA, rB, u, T = lat.moments()
    ref = oracle_run(9, fl.rho_A, fl.rho_B, 1.0, 1.0, 1.3, 100)
    orho, ou, _, OT = oracle.observables(ref, 1.0, 1.0, 1.3, probe=list(fl.centre) + [16.0])
    assert maxabs(rA, orho[0]) <= TOL and maxabs(rB, orho[1]) <= TOL
    assert maxabs(u, ou) <= TOL
    for k in ("n_in", "n_out", "n_phi_pos"):
        assert T[k] == OT[k], k
    for k in ("mass_A", "mass_B", "p_in", "p_out", "rhoA_in", "rhoA_out", "R_eff", "ke"):
        assert abs(T[k] - OT[k]) <= 1e-12 * max(1.0, abs(OT[k])), k
    assert abs(T["dp"] - OT["dp"]) <= 1e-12
    assert abs(T["max_u"] - OT["max_u"]) <= 1e-13
    for k in ("mom_x", "mom_y", "mom_z"):
        assert abs(T[k] - OT[k]) <= 1e-11 and abs(T[k]) <= 1e-11
    assert T["n_nonfinite"] == 0 and T["step"] == 100


def test_observables_3d_with_body_force():
    fl = sc_inputs.drop(24, 20, 16, radius=5, seed=7)
    say("D3Q19 24x20x16 observables with body force, 30 steps")
    lat, f = gpu_run(19, fl.rho_A, fl.rho_B, 0.8, 1.1, 1.2, 30, body_A=1e-3)
    lat.set_probe(*fl.centre, 5.0)
    rA, rB, u, T = lat.moments()
    ref = oracle_run(19, fl.rho_A, fl.rho_B, 0.8, 1.1, 1.2, 30, body_A=1e-3)
    orho, ou, _, OT = oracle.observables(ref, 0.8, 1.1, 1.2, probe=list(fl.centre) + [5.0],
                                         body_A=1e-3)
    assert maxabs(u, ou) <= TOL
    assert T["n_in"] == OT["n_in"] and T["n_out"] == OT["n_out"]
    assert abs(T["dp"] - OT["dp"]) <= 1e-12


def test_population_round_trip_and_restart():
    """set_populations(oracle state) -> get_populations is exact in FP64, and a
    step from there matches the oracle's next step (checkpoint / resume)."""
    fl = sc_inputs.drop(40, 30, 1, radius=8, seed=3)
    f0 = oracle.run(oracle.init(9, fl.rho_A, fl.rho_B), 1.0, 1.0, 1.3, 17)
    from paper_1112_5547_amd import Lattice
    say("D2Q9 40x30 set/get populations + 5 steps")
    lat = Lattice(9, 40, 30, 1, tau_A=1.0, tau_B=1.0, G=1.3)
    lat.set_populations(f0)
    assert np.array_equal(lat.get_populations(), f0)
    lat.step(5)
    assert maxabs(lat.get_populations(), oracle.run(f0, 1.0, 1.0, 1.3, 5)) <= TOL


def test_split_run_equals_single_run_bitwise():
    """100 + 100 steps through a population checkpoint equals 200 steps."""
    from paper_1112_5547_amd import Lattice
    fl = sc_inputs.drop(48, 48, 1, radius=12, seed=4)
    say("D2Q9 48x48 checkpoint resume, 200 steps")
    a = Lattice(9, 48, 48, tau_A=1.0, G=1.3).init(fl.rho_A, fl.rho_B)
    a.step(200)
    b = Lattice(9, 48, 48, tau_A=1.0, G=1.3).init(fl.rho_A, fl.rho_B)
    b.step(100)
    ck = b.get_populations()
    c = Lattice(9, 48, 48, tau_A=1.0, G=1.3)
    c.set_populations(ck)
    c.step(100)
    assert np.array_equal(a.get_populations(), c.get_populations())


def test_runs_are_deterministic():
    fl = sc_inputs.spinodal(40, 36, 20, seed=9)
    outs = []
    for k in range(2):
        say(f"D3Q19 40x36x20 determinism run {k}")
        _, f = gpu_run(19, fl.rho_A, fl.rho_B, 1.0, 1.0, 1.6, 30)
        outs.append(f)
    assert np.array_equal(outs[0], outs[1])


def test_graph_replay_equals_plain_launches():
    """Lattices below the graph threshold replay 32-step graphs; the result
    is bitwise that of plain launches (a mix of replays and single steps)."""
    from paper_1112_5547_amd import Lattice
    fl = sc_inputs.drop(64, 64, 1, radius=16, seed=1)
    say("graph replay vs plain launches, D2Q9 64x64, 77 steps")
    a = Lattice(9, 64, 64, tau_A=1.0, G=1.3).init(fl.rho_A, fl.rho_B)
    a.step(77)  # 2 replays + 13 plain steps
    b = Lattice(9, 64, 64, tau_A=1.0, G=1.3).init(fl.rho_A, fl.rho_B)
    for _ in range(77):
        b.step(1)
    assert np.array_equal(a.get_populations(), b.get_populations())
