"""The documented layout of the population buffers (lbm_sc_buffer_layout).

The raw device buffer holding the current state, read through the stride and
row pitch the library reports, equals the exported state element by element:
f_is(x, t) sits at x - c_i (pulled storage), shifted FP32 values plus
w_i rho_ref_s give the full population.  Lattices below 2^16 sites keep rows
of nx elements; larger ones pad rows to 32 elements unless nx is a multiple
of 32.  Sites past a row's nx (padding) are never written, so a step from a
state whose padding holds NaN still matches the oracle.
"""
import numpy as np
import pytest

import oracle
import sc_inputs
from gpu_common import maxabs, say

pytestmark = pytest.mark.gpu

CASES = [  # (q, nx, ny, nz, expected pitch)
    (9, 100, 70, 1, 100),        # 7,000 sites: no padding
    (9, 300, 230, 1, 320),       # 69,000 sites: rows of 300 padded to 320
    (19, 45, 40, 37, 64),        # 66,600 sites: rows of 45 padded to 64
    (19, 64, 40, 30, 64),        # 76,800 sites: rows already a multiple of 32
]


def _raw_state(lat, precision):
    """The current population buffer as one flat host array."""
    import torch
    b0, b1, cur, stride, pitch = lat.buffer_layout
    buf = (b0, b1)[cur]
    off = buf - lat._arena.data_ptr()
    esz = 8 if precision == "fp64" else 4
    n = 2 * lat.q * stride * esz
    raw = lat._arena[off:off + n].view(torch.float64 if esz == 8 else torch.float32)
    return raw.cpu().numpy(), stride, pitch


@pytest.mark.parametrize("precision", ["fp64", "fp32_shifted"])
@pytest.mark.parametrize("case", CASES)
def test_raw_buffers_follow_the_reported_layout(case, precision):
    from paper_1112_5547_amd import Lattice
    q, nx, ny, nz, want_pitch = case
    say(f"layout D{'2Q9' if q == 9 else '3Q19'} {nx}x{ny}x{nz} {precision}")
    fl = sc_inputs.spinodal(nx, ny, nz, seed=21)
    lat = Lattice(q, nx, ny, nz, tau_A=1.0, G=1.5, precision=precision)
    lat.init(fl.rho_A, fl.rho_B)
    lat.step(3)
    f = lat.get_populations()                       # [s][i][z][y][x], full values
    raw, stride, pitch = _raw_state(lat, precision)
    rho_ref = lat.rho_ref
    lat.close()
    assert pitch == want_pitch
    assert stride >= pitch * ny * nz
    c, w = oracle.lattice(q)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for s in range(2):
        for i in range(q):
            xs = (x - c[i, 0]) % nx
            ys = (y - c[i, 1]) % ny
            zs = (z - c[i, 2]) % nz
            e = (zs * ny + ys) * pitch + xs
            got = raw[(s * q + i) * stride + e].astype(np.float64)
            if precision != "fp64":
                got = got + w[i] * rho_ref[s]
            assert np.array_equal(got, f[s, i]), (s, i)


def test_padding_is_never_read():
    """Padding columns filled with NaN before a step leave the result equal
    to the oracle's (a read of any padding element would spread the NaN)."""
    import torch
    from paper_1112_5547_amd import Lattice
    q, nx, ny, nz = 19, 45, 40, 37
    say("layout: NaN in the row padding, 4 steps against the oracle")
    fl = sc_inputs.spinodal(nx, ny, nz, seed=22)
    lat = Lattice(q, nx, ny, nz, tau_A=1.0, G=1.5)
    lat.init(fl.rho_A, fl.rho_B)
    b0, b1, cur, stride, pitch = lat.buffer_layout
    assert pitch > nx
    torch.cuda.synchronize()
    for buf in (b0, b1):
        off = buf - lat._arena.data_ptr()
        arr = lat._arena[off:off + 2 * q * stride * 8].view(torch.float64)
        rows = arr[:2 * q * stride].view(2 * q, stride)[:, :pitch * ny * nz]
        rows.view(2 * q, ny * nz, pitch)[:, :, nx:] = float("nan")
    torch.cuda.synchronize()
    lat.step(4)
    f = lat.get_populations()
    lat.close()
    want = oracle.run(oracle.init(q, fl.rho_A, fl.rho_B), 1.0, 1.0, 1.5, 4)
    assert np.isfinite(f).all()
    assert maxabs(f, want) <= 1e-12
