"""Error paths of the C ABI on a live handle: each misuse returns its status
(raised by the binding as LbmError) and leaves the handle usable; a lattice
that diverges is reported as LBM_ENONFINITE by the FP64 reductions.

Every case here is refused by the host-side checks before any kernel runs,
or (divergence) runs ordinary kernels on non-finite values."""
import numpy as np
import pytest

import oracle
import sc_inputs
from gpu_common import say

pytestmark = pytest.mark.gpu


def _status(fn, *a, **k):
    from paper_1112_5547_amd import LbmError
    with pytest.raises(LbmError) as e:
        fn(*a, **k)
    return e.value.status


def test_call_order_and_argument_errors_leave_the_handle_usable():
    from paper_1112_5547_amd import Lattice, _abi
    say("error paths: D2Q9 40x24")
    fl = sc_inputs.drop(40, 24, 1, radius=6, seed=3)
    lat = Lattice(9, 40, 24, tau_A=0.9, G=1.3)
    # nothing to step, read or export before init
    assert _status(lat.step, 1) == _abi.LBM_ESTATE
    assert _status(lat.moments) == _abi.LBM_ESTATE
    assert _status(lat.get_populations) == _abi.LBM_ESTATE
    # densities must be positive and finite
    bad = fl.rho_A.copy()
    bad[0, 3, 5] = -0.1
    assert _status(lat.init, bad, fl.rho_B) == _abi.LBM_EINVAL
    bad[0, 3, 5] = np.nan
    assert _status(lat.init, bad, fl.rho_B) == _abi.LBM_EINVAL
    lat.init(fl.rho_A, fl.rho_B)
    # negative step counts, unknown tiles and a non-finite probe are refused
    assert _status(lat.step, -1) == _abi.LBM_EINVAL
    before = lat.kernel
    assert _status(lat.set_kernel, 0, 48, 1, 4) == _abi.LBM_EINVAL
    assert lat.kernel == before
    assert _status(lat.set_probe, 20.0, np.nan, 0.0, 6.0) == _abi.LBM_EINVAL
    f = lat.get_populations()
    g = f.copy()
    g[1, 4, 0, 2, 7] = np.inf
    assert _status(lat.set_populations, g) == _abi.LBM_EINVAL
    # after all of that the handle still steps exactly like the oracle
    lat.step(20)
    ref = oracle.run(oracle.init(9, fl.rho_A, fl.rho_B), 0.9, 0.9, 1.3, 20)
    assert np.abs(lat.get_populations() - ref).max() <= 1e-12
    lat.close()


def test_divergence_is_reported_as_nonfinite():
    """tau = 0.52 with G = 6 is far outside the stable range: the state turns
    non-finite within 50 steps (the oracle does too); the FP64 reductions flag
    it and the binding raises unless asked to return the totals."""
    from paper_1112_5547_amd import Lattice, _abi
    fl = sc_inputs.spinodal(32, 32, 1, seed=5)
    ref = oracle.run(oracle.init(9, fl.rho_A, fl.rho_B), 0.52, 0.52, 6.0, 50)
    assert not np.isfinite(ref).all()
    for precision in ("fp64", "fp32_shifted"):
        say(f"divergence {precision}")
        lat = Lattice(9, 32, 32, tau_A=0.52, G=6.0, precision=precision)
        lat.init(fl.rho_A, fl.rho_B)
        lat.step(50)
        assert _status(lat.moments) == _abi.LBM_ENONFINITE
        T = lat.totals(allow_nonfinite=True)
        assert T["n_nonfinite"] > 0
        lat.close()
