"""Batched launches against the oracle, and alone against in the mix.

Every batched member is compared with the FP64 CPU oracle run from the same
seeded fields (Sec. 2.1 step by step): populations within 1e-12 in FP64 and
2e-6 in FP32 shifted storage.  Every batch mode also runs the same per-site
device code as a single-lattice launch, so the alone-vs-in-the-mix comparison
is exact equality, for FP64 and FP32-shifted members, D2Q9 and D3Q19 in one
launch, uneven sizes, members with different step counts, members joining
mid-run, every compiled batch block shape with and without march-chunk
overrides, and groups of D2Q9 members only at every block size.
"""
import numpy as np
import pytest

import oracle
import sc_inputs
from gpu_common import maxabs, say

TOL = {"fp64": 1e-12, "fp32_shifted": 2e-6}
_ORACLE = {}


def _oracle(spec, seed):
    """Oracle populations of a member after its steps (cached per spec, seed)."""
    key = (spec, seed)
    if key not in _ORACLE:
        q, nx, ny, nz, tau, G, steps, kind = spec
        fl = _fields(q, nx, ny, nz, kind, seed)
        _ORACLE[key] = oracle.run(oracle.init(q, fl.rho_A, fl.rho_B), tau, tau, G, steps,
                                  all_cores=True)
    return _ORACLE[key]

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
    for k, (lat, spec, ref) in enumerate(zip(lats, SPECS, solo)):
        assert lat.steps_done == spec[6]
        b.remove(lat)
        f = lat.get_populations()
        assert np.array_equal(f, ref), spec
        err = maxabs(f, _oracle(spec, 100 + k))
        assert err <= TOL[precision], (spec, err)
    b.close()


# every block shape the batch kernels are compiled for (tx9 = block size,
# tx19 x ty19 the D3Q19 tile), each with its default march chunks and with
# overridden ones
BATCH_CFGS = [(256, 64, 4), (256, 32, 8), (256, 16, 16), (128, 32, 4), (512, 64, 8),
              (512, 32, 16)]


# groups without D3Q19 members (every epoch of such a batch) at each block
# size; one D3Q19 tile per block size
D2Q9_TILES = {128: (32, 4), 256: (64, 4), 512: (64, 8)}


@pytest.mark.parametrize("nt", sorted(D2Q9_TILES))
@pytest.mark.parametrize("precision", ["fp64", "fp32_shifted"])
def test_d2q9_only_batch_against_solo_and_oracle(nt, precision):
    from paper_1112_5547_amd import Batch
    members = [(k, spec) for k, spec in enumerate(SPECS) if spec[0] == 9]
    solo = []
    for k, spec in members:
        say(f"solo {spec} {precision}")
        lat = _make(spec, 100 + k, precision)
        lat.step(spec[6])
        solo.append(lat.get_populations())
        lat.close()
    say(f"D2Q9-only batch, block {nt}, {precision}")
    b = Batch()
    b.set_tiles(nt, *D2Q9_TILES[nt], 0, 0)
    lats = [_make(spec, 100 + k, precision) for k, spec in members]
    for lat, (_, spec) in zip(lats, members):
        assert b.add(lat, spec[6])
    for _ in range(10):
        b.run(16, "fused")
        if len(b.poll()) == len(lats):
            break
    for lat, (k, spec), ref in zip(lats, members, solo):
        assert lat.steps_done == spec[6]
        b.remove(lat)
        f = lat.get_populations()
        assert np.array_equal(f, ref), spec
        err = maxabs(f, _oracle(spec, 100 + k))
        assert err <= TOL[precision], (spec, err)
        lat.close()
    b.close()


@pytest.mark.parametrize("cfg", BATCH_CFGS)
@pytest.mark.parametrize("mbs", [(0, 0), (5, 3)])
@pytest.mark.parametrize("mode", ["fused", "persistent"])
def test_every_batch_block_shape_against_oracle(cfg, mbs, mode):
    from paper_1112_5547_amd import Batch
    precision = "fp32_shifted" if cfg[0] != 512 else "fp64"
    say(f"batch tiles {cfg} mb {mbs} mode={mode} {precision}")
    b = Batch()
    b.set_tiles(cfg[0], cfg[1], cfg[2], mbs[0], mbs[1])
    lats = [_make(spec, 100 + k, precision) for k, spec in enumerate(SPECS)]
    for lat, spec in zip(lats, SPECS):
        assert b.add(lat, spec[6])
    for _ in range(10):
        b.run(16, mode)
        if len(b.poll()) == len(lats):
            break
    for k, (lat, spec) in enumerate(zip(lats, SPECS)):
        assert lat.steps_done == spec[6]
        b.remove(lat)
        err = maxabs(lat.get_populations(), _oracle(spec, 100 + k))
        assert err <= TOL[precision], (spec, err)
        lat.close()
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


def test_persistent_barrier_give_up_is_reported():
    """A spin limit of one poll makes the first block that waits at a grid
    barrier give up: every block leaves the kernel (the give-up flag is
    checked at every poll), poll reports LBM_ETIMEOUT, the members are failed
    and only removal and destroy are accepted; a new batch then runs normally."""
    from paper_1112_5547_amd import Batch, LbmError
    from paper_1112_5547_amd._abi import LBM_ETIMEOUT
    say("persistent batch with a one-poll barrier spin limit")
    b = Batch()
    b.set_spin_limit(1)
    lats = [_make(spec, 100 + k, "fp32_shifted") for k, spec in enumerate(SPECS)]
    for lat, spec in zip(lats, SPECS):
        assert b.add(lat, spec[6])
    b.run(16, "persistent")
    with pytest.raises(LbmError) as e:
        b.poll()
    assert e.value.status == LBM_ETIMEOUT
    with pytest.raises(LbmError) as e:
        lats[0].step(1)
    assert e.value.status == LBM_ETIMEOUT
    for lat in lats:
        with pytest.raises(LbmError) as e:
            b.remove(lat)
        assert e.value.status == LBM_ETIMEOUT
        lat.close()
    with pytest.raises(LbmError):
        b.close()
    say("fresh persistent batch after the give-up")
    b2 = Batch()
    lat = _make(SPECS[0], 100, "fp32_shifted")
    b2.add(lat, SPECS[0][6])
    while not b2.poll():
        b2.run(16, "persistent")
    b2.remove(lat)
    assert maxabs(lat.get_populations(), _oracle(SPECS[0], 100)) <= TOL["fp32_shifted"]
    b2.close()
