"""Batched launches give each lattice bitwise the result it has alone.

Every batch mode runs the same per-site device code as a single-lattice
launch, so the alone-vs-in-the-mix comparison is exact equality, for FP64
and FP32-shifted members, D2Q9 and D3Q19 in one launch, uneven sizes,
members with different step counts and members joining mid-run.
"""
import numpy as np
import pytest

import sc_inputs
from gpu_common import say

pytestmark = pytest.mark.gpu

SPECS = [  # (q, nx, ny, nz, tau, G, steps, kind)
    (9, 64, 64, 1, 1.0, 1.3, 50, "drop"),
    (9, 100, 80, 1, 0.7, 1.5, 37, "drop"),
    (19, 24, 20, 18, 1.0, 1.6, 45, "spinodal"),
    (9, 33, 200, 1, 1.2, 1.25, 50, "drop"),
    (19, 16, 16, 16, 0.9, 1.3, 21, "drop"),
    # above 2^16 sites with N not a multiple of 32: padded array strides
    (9, 300, 230, 1, 0.8, 1.4, 23, "drop"),
    (19, 42, 41, 40, 1.1, 1.5, 9, "spinodal"),
]


def _fields(q, nx, ny, nz, kind, seed):
    if kind == "drop":
        return sc_inputs.drop(nx, ny, nz, radius=min(nx, ny, max(nz, 8)) / 4, seed=seed)
    return sc_inputs.spinodal(nx, ny, nz, seed=seed)


def _make(spec, seed, precision):
    from paper_1112_5547_amd import Lattice
    q, nx, ny, nz, tau, G, steps, kind = spec
    fl = _fields(q, nx, ny, nz, kind, seed)
    lat = Lattice(q, nx, ny, nz, tau_A=tau, G=G, precision=precision)
    lat.init(fl.rho_A, fl.rho_B)
    return lat


@pytest.mark.parametrize("precision", ["fp64", "fp32_shifted"])
@pytest.mark.parametrize("mode", ["per_lattice", "fused", "persistent"])
def test_batch_equals_solo_bitwise(mode, precision):
    from paper_1112_5547_amd import Batch
    solo = []
    for k, spec in enumerate(SPECS):
        say(f"solo {spec} {precision}")
        lat = _make(spec, 100 + k, precision)
        lat.step(spec[6])
        solo.append(lat.get_populations())
    say(f"batch mode={mode} {precision}")
    b = Batch()
    lats = [_make(spec, 100 + k, precision) for k, spec in enumerate(SPECS)]
    for lat, spec in zip(lats, SPECS):
        assert b.add(lat, spec[6])
    done = []
    for _ in range(10):
        b.run(16, mode)
        done = b.poll()
        if len(done) == len(lats):
            break
    assert len(done) == len(lats)
    for lat, spec, ref in zip(lats, SPECS, solo):
        assert lat.steps_done == spec[6]
        b.remove(lat)
        assert np.array_equal(lat.get_populations(), ref), spec
    b.close()


def test_members_joining_mid_run_and_budget():
    from paper_1112_5547_amd import Batch, Lattice
    say("batch join mid-run + budget, fp32_shifted persistent")
    first = _make(SPECS[0], 7, "fp32_shifted")
    late = _make(SPECS[2], 8, "fp32_shifted")
    budget = first.nbytes + late.nbytes
    b = Batch(hbm_budget=budget)
    assert b.add(first, 40)
    big = Lattice(9, 512, 512, tau_A=1.0, G=1.3, precision="fp32_shifted")
    fl = sc_inputs.drop(512, 512, 1, radius=64, seed=1)
    big.init(fl.rho_A, fl.rho_B)
    assert not b.add(big, 10)          # over budget: refused, nothing queued
    b.run(16, "persistent")
    b.poll()
    assert b.add(late, 30)
    while len(b.poll()) < 2:
        b.run(16, "persistent")
    for lat in (first, late):
        b.remove(lat)
    ref_a = _make(SPECS[0], 7, "fp32_shifted")
    ref_a.step(40)
    ref_b = _make(SPECS[2], 8, "fp32_shifted")
    ref_b.step(30)
    assert np.array_equal(first.get_populations(), ref_a.get_populations())
    assert np.array_equal(late.get_populations(), ref_b.get_populations())
    assert b.stats()["members"] == 0
    b.close()


def test_member_cannot_step_alone_while_batched():
    from paper_1112_5547_amd import Batch, LbmError
    say("batched member refuses solo step")
    lat = _make(SPECS[0], 1, "fp64")
    b = Batch()
    b.add(lat, 5)
    with pytest.raises(LbmError):
        lat.step(1)
    b.run(5, "fused")
    b.poll()
    b.remove(lat)
    lat.step(1)
    b.close()
