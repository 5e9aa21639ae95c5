"""The largest lattices one MI355X holds, checked through periodicity.

A state that repeats with period p along every axis evolves exactly as the
p^3 lattice does, site for site and operation for operation.  So a lattice of
hundreds of millions of sites, tiled from a seeded 10^3 cell, must give at
every site bitwise the FP64 densities and velocities of the 10^3 lattice
(which is itself checked against the oracle).  This reaches population byte
offsets beyond 2^31 (FP64, 300M sites, 200 GB) and the site-count limit class
(FP32 shifted, 525M sites, 185 GB), where a 32-bit signed or truncated
offset anywhere in the step, init or observables would show.  Only density
and velocity fields (5 doubles per site) come back to the host."""
import numpy as np
import pytest

import oracle
import sc_inputs
from gpu_common import say

pytestmark = pytest.mark.gpu

P = 10  # period of the tiled cell


def _need_hbm(nbytes):
    import torch
    torch.cuda.empty_cache()            # arenas of earlier tests held by the allocator
    free, _ = torch.cuda.mem_get_info(0)
    if free < nbytes + (8 << 30):
        pytest.skip(f"needs {nbytes / 1e9:.0f} GB of free device memory, {free / 1e9:.0f} GB free")


def _run(nx, ny, nz, precision, tau_A, tau_B, G, steps, rho_ref):
    from paper_1112_5547_amd import Lattice
    cell = sc_inputs.spinodal(P, P, P, seed=41)
    small = Lattice(19, P, P, P, tau_A=tau_A, tau_B=tau_B, G=G, precision=precision,
                    rho_ref=rho_ref)
    small.init(cell.rho_A, cell.rho_B)
    small.step(steps)
    sA, sB, su, sT = small.moments()
    f_small = small.get_populations()
    small.close()

    reps = (nz // P, ny // P, nx // P)
    lat = Lattice(19, nx, ny, nz, tau_A=tau_A, tau_B=tau_B, G=G, precision=precision,
                  rho_ref=rho_ref)
    rA = np.tile(cell.rho_A, reps)
    rB = np.tile(cell.rho_B, reps)
    lat.init(rA, rB)
    del rA, rB
    lat.step(steps)
    bA, bB, bu, bT = lat.moments()
    lat.close()

    def same(big, ref):
        # every P^3 cell of the big field equals the small field
        v = big.reshape(reps[0], P, reps[1], P, reps[2], P)
        r = ref.reshape(1, P, 1, P, 1, P)
        return bool(np.array_equal(v, np.broadcast_to(r, v.shape)))

    assert same(bA, sA)
    assert same(bB, sB)
    for a in range(3):
        assert same(bu[a], su[a])
    cells = reps[0] * reps[1] * reps[2]
    assert abs(bT["mass_A"] - cells * sT["mass_A"]) <= 1e-12 * abs(bT["mass_A"])
    return f_small, cell


def test_fp64_offsets_beyond_2_31():
    nx, ny, nz = 680, 670, 660          # 300.7M sites: populations reach 2.4 GB offsets
    from paper_1112_5547_amd import bytes_needed
    _need_hbm(bytes_needed(19, nx, ny, nz, "fp64"))
    say(f"max-size fp64 {nx}x{ny}x{nz}, 6 steps")
    f_small, cell = _run(nx, ny, nz, "fp64", 1.0, 0.9, 1.6, 6, None)
    ref = oracle.run(oracle.init(19, cell.rho_A, cell.rho_B), 1.0, 0.9, 1.6, 6)
    assert np.abs(f_small - ref).max() <= 1e-12


def test_fp32_shifted_at_the_site_count_limit():
    nx, ny, nz = 810, 810, 800          # 524.9M sites (limit 2^29 - 2112)
    from paper_1112_5547_amd import bytes_needed
    _need_hbm(bytes_needed(19, nx, ny, nz, "fp32_shifted"))
    say(f"max-size fp32_shifted {nx}x{ny}x{nz}, 6 steps")
    _run(nx, ny, nz, "fp32_shifted", 1.0, 0.9, 1.6, 6, (0.5, 0.5))
