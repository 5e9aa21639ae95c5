"""The allocation-free batch run (lbm_batch_run_noalloc) against lbm_batch_run.

Both launch the same fused batch kernels; the allocation-free one takes its
descriptor table and work list from the library's fixed per-GPU scratch array.
Two calls in a row through the C ABI, the second with a smaller batch (the
scratch keeps the first call's larger tables): every member equals the
allocating run bitwise and the oracle within the precision's bound.  A group
beyond the scratch limits is refused with LBM_ETOOBIG before anything runs.
"""
import numpy as np
import pytest

import oracle
import sc_inputs
from gpu_common import maxabs, say

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32_shifted": 2e-6}

BIG = [  # (q, nx, ny, nz, tau, G, steps, kind, precision)
    (9, 96, 80, 1, 1.0, 1.3, 40, "drop", "fp32_shifted"),
    (19, 24, 20, 18, 1.0, 1.6, 33, "spinodal", "fp32_shifted"),
    (9, 300, 230, 1, 0.8, 1.4, 21, "drop", "fp32_shifted"),
    (9, 64, 64, 1, 1.2, 1.25, 40, "drop", "fp64"),
    (19, 20, 20, 20, 0.9, 1.3, 27, "drop", "fp64"),
]
SMALL = [
    (9, 40, 36, 1, 1.1, 1.3, 25, "drop", "fp32_shifted"),
    (19, 12, 10, 8, 1.0, 1.6, 19, "spinodal", "fp64"),
]


def _fields(spec, seed):
    q, nx, ny, nz, tau, G, steps, kind, prec = spec
    if kind == "drop":
        return sc_inputs.drop(nx, ny, nz, radius=min(nx, ny, max(nz, 8)) / 4, seed=seed)
    return sc_inputs.spinodal(nx, ny, nz, seed=seed)


def _make(spec, seed):
    from paper_1112_5547_amd import Lattice
    q, nx, ny, nz, tau, G, steps, kind, prec = spec
    fl = _fields(spec, seed)
    lat = Lattice(q, nx, ny, nz, tau_A=tau, G=G, precision=prec)
    lat.init(fl.rho_A, fl.rho_B)
    return lat


def _run(specs, seed0, noalloc, epoch=16):
    from paper_1112_5547_amd import Batch
    b = Batch()
    lats = [_make(spec, seed0 + k) for k, spec in enumerate(specs)]
    for lat, spec in zip(lats, specs):
        assert b.add(lat, spec[6])
    for _ in range(10):
        if noalloc:
            b.run_noalloc(epoch, "fused")
        else:
            b.run(epoch, "fused")
        if len(b.poll()) == len(lats):
            break
    out = []
    for lat, spec in zip(lats, specs):
        assert lat.steps_done == spec[6]
        b.remove(lat)
        out.append(lat.get_populations())
        lat.close()
    b.close()
    return out


@pytest.mark.parametrize("specs,seed0", [(BIG, 200), (SMALL, 300)], ids=["first", "smaller"])
def test_noalloc_run_equals_allocating_run(specs, seed0):
    say(f"no-alloc batch run: {len(specs)} members (allocating run first)")
    ref = _run(specs, seed0, noalloc=False)
    say(f"no-alloc batch run: {len(specs)} members (allocation-free run)")
    got = _run(specs, seed0, noalloc=True)
    for k, (spec, a, r) in enumerate(zip(specs, got, ref)):
        assert np.array_equal(a, r), spec
        q, nx, ny, nz, tau, G, steps, kind, prec = spec
        fl = _fields(spec, seed0 + k)
        want = oracle.run(oracle.init(q, fl.rho_A, fl.rho_B), tau, tau, G, steps)
        assert maxabs(a, want) <= TOL[prec], spec


def test_noalloc_refuses_a_group_beyond_the_scratch():
    from paper_1112_5547_amd import Batch, LbmError, Lattice
    from paper_1112_5547_amd._abi import LBM_ETOOBIG
    say("no-alloc batch run: 1025 members (over the limit)")
    b = Batch()
    lats = []
    for k in range(1025):
        lat = Lattice(9, 4, 4, 1, tau_A=1.0, G=1.0, precision="fp32_shifted")
        lat.init(np.full((1, 4, 4), 0.6), np.full((1, 4, 4), 0.4))
        b.add(lat, 2)
        lats.append(lat)
    with pytest.raises(LbmError) as e:
        b.run_noalloc(2, "fused")
    assert e.value.status == LBM_ETOOBIG
    assert all(lat.steps_done == 0 for lat in lats)
    with pytest.raises(LbmError):
        b.run_noalloc(2, "persistent")
    for lat in lats:
        b.remove(lat)
        lat.close()
    b.close()
