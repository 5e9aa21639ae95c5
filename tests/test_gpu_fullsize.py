"""Full-size checks in the benchmark's launch configuration.

At 256^3 D3Q19 a full oracle step takes about half a minute, so the step is
checked on sampled sites the oracle computes one by one (oracle.step_sites),
and the run over many steps through properties that hold at any size (mass
per species conserved to roundoff, lattice momentum stays zero).  The 128^3
drop is checked the same way on a state the GPU evolved for 800 steps, where
the interface carries the largest gradients, and so are the benchmark's batch of
64 D2Q9 lattices in its fused launch and the largest lattices of its served
job stream (ragged tiles at full size).
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
@pytest.mark.parametrize("forcing,tau_minus", [("shift", None), ("guo", None),
                                               ("shift", (0.8, 0.8))])
def test_256cube_one_step_sampled(spinodal256, precision, tol, forcing, tau_minus):
    """The benchmark's step kernels (the tuned configuration bench.py times,
    for the velocity shift, Guo forcing and two relaxation times) against the
    oracle's one-site-at-a-time step."""
    from paper_1112_5547_amd import Lattice, autotune
    fl = spinodal256
    say(f"256^3 D3Q19 {precision} {forcing} tau- {tau_minus}: init + 1 step (bench kernel)")
    lat = Lattice(19, L, L, L, tau_A=TAU, G=G, precision=precision, forcing=forcing,
                  tau_minus=tau_minus)
    autotune.apply(lat)
    say(f"kernel {lat.kernel}")
    lat.init(fl.rho_A, fl.rho_B)
    lat.step(1)
    f = lat.get_populations().reshape(2, 19, -1)
    lat.close()
    f0 = oracle.init(19, fl.rho_A, fl.rho_B)
    sites = _sample_sites(L ** 3, 3000, 1)
    want = oracle.step_sites(f0, TAU, TAU, G, sites, forcing=forcing, tau_minus=tau_minus)
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


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_shifted", 2e-6)])
def test_128cube_drop_evolved_state_sampled(precision, tol):
    """128^3 D3Q19 drop (R = 24, tau = 1, G = 1.3, seed 2): after 800 GPU
    steps, one more GPU step equals the oracle's step from the GPU's own state
    at 3000 random sites and at every sampled site on the drop surface."""
    from paper_1112_5547_amd import Lattice
    n = 128
    fl = sc_inputs.drop(n, n, n, radius=24, seed=2)
    say(f"128^3 D3Q19 drop {precision}: 800 steps, then one step against the oracle")
    lat = Lattice(19, n, n, n, tau_A=1.0, G=1.3, precision=precision)
    lat.init(fl.rho_A, fl.rho_B)
    lat.set_probe(*fl.centre, 24.0)
    lat.step(800)
    f800 = lat.get_populations()
    lat.step(1)
    f801 = lat.get_populations().reshape(2, 19, -1)
    T = lat.totals()
    lat.close()
    # (the Laplace pressure still oscillates at step 800; only its finiteness is checked)
    assert T["n_nonfinite"] == 0 and np.isfinite(T["dp"])
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    cx, cy, cz = fl.centre
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2).ravel()
    surface = np.flatnonzero(np.abs(r - 24.0) < 0.5)[::7]
    rng = np.random.default_rng(5)
    sites = np.unique(np.concatenate([rng.integers(0, n ** 3, 3000), surface])).astype(np.int64)
    # the interface is where the state moved most: it is not the initial profile any more
    rho_A = f800[0].sum(axis=0).ravel()
    assert np.abs(rho_A[surface] - fl.rho_A.ravel()[surface]).max() > 1e-4
    want = oracle.step_sites(f800, 1.0, 1.0, 1.3, sites)
    got = f801[:, :, sites].transpose(2, 0, 1)
    assert float(np.abs(got - want).max()) <= tol


def _batch_sites(nx, ny, tx, rng, k=120):
    """Random sites plus the lattice edges, the tile edges along x and the
    march-chunk edges along y (chunks of 8 rows) of an nx x ny lattice."""
    xs = [0, 1, nx - 2, nx - 1] + [x for x in (tx - 1, tx, tx + 1) if x < nx]
    ys = [0, 7, 8, ny // 2, ny - 1]
    edge = [y * nx + x for y in ys for x in xs]
    return np.unique(np.concatenate([rng.integers(0, nx * ny, k), edge])).astype(np.int64)


@pytest.mark.parametrize("tiles", [(256, 32, 8), (512, 64, 8)])
def test_batch_of_64_lattices_sampled(tiles):
    """The batch leg's 64 D2Q9 drop lattices (64^2-512^2, 6.87 M sites, FP32
    shifted, per-lattice tau and G) in the fused launch, at the block shapes
    its autotuner picks: after 20 batched steps, one more batched step equals
    the oracle's one-site step from the batch's own state at sampled sites of
    every member."""
    from paper_1112_5547_amd import Batch, Lattice
    jobs = sc_inputs.batch_jobs(64, seed=4)
    say(f"batch of 64 D2Q9 lattices, tiles {tiles}: 20 fused steps, then one more")
    lats = []
    for j in jobs:
        lat = Lattice(9, j.nx, j.ny, 1, tau_A=j.tau, G=j.G, precision="fp32_shifted")
        fl = j.fields()
        lat.init(fl.rho_A, fl.rho_B)
        lats.append(lat)
    b = Batch()
    b.set_tiles(*tiles, 0, 0)
    for lat in lats:
        assert b.add(lat, 20)
    b.run(20, "fused")
    assert len(b.poll()) == len(lats)
    rng = np.random.default_rng(7)
    wants = []
    for lat, j in zip(lats, jobs):
        b.remove(lat)
        f20 = lat.get_populations()
        sites = _batch_sites(j.nx, j.ny, tiles[0], rng)
        wants.append((sites, oracle.step_sites(f20, j.tau, j.tau, j.G, sites)))
    for lat in lats:
        assert b.add(lat, 1)
    b.run(1, "fused")
    assert len(b.poll()) == len(lats)
    worst = 0.0
    for lat, j, (sites, want) in zip(lats, jobs, wants):
        b.remove(lat)
        assert lat.steps_done == 21
        f21 = lat.get_populations().reshape(2, 9, -1)
        got = f21[:, :, sites].transpose(2, 0, 1)
        worst = max(worst, float(np.abs(got - want).max()))
        lat.close()
    b.close()
    assert worst <= 2e-6, worst


@pytest.mark.parametrize("rank", [0, 1])
def test_largest_served_lattices_sampled(rank):
    """The two largest D3Q19 jobs of the served stream (seed 5: a 250^3 drop
    and a 249^3 spinodal, FP32 shifted), built as the server builds them (its
    backend, with the autotuned solo kernel).  Their last tiles are ragged in
    x and y: after 10 steps, one more step equals the oracle's one-site step
    from the GPU's own state at random sites and on the tile, chunk and
    lattice edges."""
    from paper_1112_5547_amd.serve import GpuBackend
    jobs = sorted((j for j in sc_inputs.serving_jobs(200, seed=5) if j.lattice == 19),
                  key=lambda j: -j.sites)
    job = jobs[rank]
    n = job.nx
    say(f"served {n}^3 {job.kind} fp32_shifted: 10 steps, then one step against the oracle")
    be = GpuBackend("fp32_shifted")
    lat = be.make_lattice(job)
    _, tx, ty, mb = lat.kernel
    lat.step(10)
    f10 = lat.get_populations()
    rng = np.random.default_rng(11)
    xs = sorted({0, n - 1} | {x for k in range(1, n // tx + 1) for x in (k * tx - 1, k * tx)
                              if x < n})
    ys = sorted({0, n - 1} | {y for k in range(1, n // ty + 1) for y in (k * ty - 1, k * ty)
                              if y < n})
    zs = sorted({0, n - 1} | {z for k in range(1, n // mb + 1) for z in (k * mb - 1, k * mb)
                              if z < n})
    edge = [(z * n + y) * n + x for z in zs[:6] + zs[-2:] for y in ys[:2] + ys[-3:]
            for x in xs]
    sites = np.unique(np.concatenate([rng.integers(0, n ** 3, 3000), edge])).astype(np.int64)
    want = oracle.step_sites(f10, job.tau, job.tau, job.G, sites)
    del f10
    lat.step(1)
    f11 = lat.get_populations().reshape(2, 19, -1)
    be.release(lat)
    got = f11[:, :, sites].transpose(2, 0, 1)
    assert float(np.abs(got - want).max()) <= 2e-6
