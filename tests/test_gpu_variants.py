"""Every kernel variant, tile shape and march chunk advances a lattice bitwise
the same: the device code is compiled without implicit contraction and writes
its fused multiply-adds out, so the rounding of each site update does not
depend on the launch form.  The served-job and batch equalities rest on this."""
import numpy as np
import pytest

import sc_inputs
from gpu_common import gpu_run, say

pytestmark = pytest.mark.gpu

D2 = [(0, 64, 1, 16), (0, 256, 1, 5), (1, 64, 1, 4), (2, 64, 1, 16), (2, 128, 1, 7),
      (3, 64, 1, 16)]
D3 = [(0, 64, 4, 8), (0, 32, 8, 3), (0, 16, 16, 32), (1, 64, 4, 4), (2, 64, 4, 8),
      (2, 32, 8, 5), (3, 64, 4, 8), (3, 32, 16, 6)]


@pytest.mark.parametrize("precision", ["fp64", "fp32_shifted"])
@pytest.mark.parametrize("q,shape,kernels", [(9, (1, 142, 130), D2), (19, (30, 36, 40), D3)])
def test_all_variants_agree_bitwise(q, shape, kernels, precision):
    nz, ny, nx = shape
    fl = sc_inputs.drop(nx, ny, nz, radius=nx / 5, seed=3)
    ref = None
    for k in kernels:
        say(f"variants q={q} {shape} {precision} kernel {k}")
        lat, f = gpu_run(q, fl.rho_A, fl.rho_B, 0.9, 1.1, 1.4, 40, precision=precision, kernel=k)
        lat.close()
        if ref is None:
            ref = f
        else:
            assert np.array_equal(f, ref), (k, float(np.abs(f.astype(float) - ref).max()))
