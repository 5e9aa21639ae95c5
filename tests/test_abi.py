"""The C-ABI library loads on a machine without a GPU and exports every
function include/lbm_sc.h declares; host-only entry points validate their
arguments.  No kernel is launched here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm_sc.h")
LIB = os.path.join(ROOT, "paper_1112_5547_amd", "liblbm_sc.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_(?:sc|batch)_\w+)\s*\(", text)))


def _lib():
    if not os.path.exists(LIB):
        from paper_1112_5547_amd import build
        build.build()
    from paper_1112_5547_amd import _abi
    return _abi.lib()


def test_header_declares_the_core_calls():
    names = _declared()
    for core in ("lbm_sc_create", "lbm_sc_init", "lbm_sc_step", "lbm_sc_moments",
                 "lbm_sc_destroy", "lbm_batch_run"):
        assert core in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_1112_5547_amd import _abi
    bound = {n for n, _, _ in _abi.SIGNATURES}
    assert bound == set(_declared())


def test_params_validation_and_sizes():
    from paper_1112_5547_amd import _abi
    L = _lib()
    p = _abi.Params()
    ok = L.lbm_sc_params_default(ctypes.byref(p), 19, 256, 256, 256, 1.0, 1.0, 1.6)
    assert ok == 0
    n = 256 ** 3
    need = L.lbm_sc_bytes_needed(ctypes.byref(p))
    assert need >= 2 * (2 * 19 * n * 8)          # two FP64 population buffers
    assert need < 2 * (2 * 19 * n * 8) * 1.2      # plus small side arrays
    p.precision = _abi.LBM_FP32_SHIFTED
    need32 = L.lbm_sc_bytes_needed(ctypes.byref(p))
    assert need32 < need
    # the forcing field sits where the C struct has it: the default fill
    # overwrites it, and an unknown scheme is rejected
    f = _abi.Params()
    f.forcing = 7
    assert L.lbm_sc_params_default(ctypes.byref(f), 9, 8, 8, 1, 1.0, 1.0, 1.0) == 0
    assert f.forcing == _abi.LBM_FORCING_SHIFT and f.body_A == 0.0
    f.forcing = _abi.LBM_FORCING_GUO
    assert L.lbm_sc_bytes_needed(ctypes.byref(f)) > 0
    f.forcing = 2
    assert L.lbm_sc_bytes_needed(ctypes.byref(f)) == 0
    # odd-part relaxation times: 0 (BGK) or > 1/2
    f.forcing = 0
    assert f.tau_minus_A == 0.0 and f.tau_minus_B == 0.0
    f.tau_minus_A, f.tau_minus_B = 0.7, 1.3
    assert L.lbm_sc_bytes_needed(ctypes.byref(f)) > 0
    f.tau_minus_B = 0.5
    assert L.lbm_sc_bytes_needed(ctypes.byref(f)) == 0
    bad = [
        (9, 8, 8, 2, 1.0, 1.0, 1.0),     # D2Q9 with nz > 1
        (19, 0, 8, 8, 1.0, 1.0, 1.0),    # empty lattice
        (9, 8, 8, 1, 0.5, 1.0, 1.0),     # tau = 1/2: zero viscosity
        (9, 8, 8, 1, 1.0, 0.4, 1.0),
        (9, 8, 8, 1, 1.0, 1.0, -0.1),    # attractive coupling not supported
        (7, 8, 8, 1, 1.0, 1.0, 1.0),     # unknown lattice
        (19, 1024, 1024, 1024, 1.0, 1.0, 1.0),  # beyond 2^29 sites
    ]
    for args in bad:
        q = _abi.Params()
        assert L.lbm_sc_params_default(ctypes.byref(q), *args) == _abi.LBM_EINVAL, args
        assert L.lbm_sc_bytes_needed(ctypes.byref(q)) == 0


def _pop_bytes(q, nx, ny, nz, es):
    """Population bytes of a handle (both buffers), from its total minus the
    side arrays (psi 2N es, rho 2N 8, u 3N 8, reduction partials)."""
    from paper_1112_5547_amd import _abi
    p = _abi.Params()
    assert _lib().lbm_sc_params_default(ctypes.byref(p), q, nx, ny, nz, 1.0, 1.0, 1.0) == 0
    if es == 4:
        p.precision = _abi.LBM_FP32_SHIFTED
    return int(_lib().lbm_sc_bytes_needed(ctypes.byref(p)))


def test_population_arrays_are_padded_and_aligned():
    """Each of the 2Q arrays of a buffer spans N rounded up to 32 elements,
    plus 2080 elements from 2^16 sites on (staggers power-of-two strides
    across HBM channels).  Checked through bytes_needed as N grows."""
    for q, es in ((9, 8), (19, 4)):
        nz = 1 if q == 9 else 2
        b32, b33, b34 = (_pop_bytes(q, n, 1, nz, es) for n in (32, 33, 34))
        block = 2 * 2 * q * 32 * es        # both buffers, 2Q arrays, 32 more elements
        side = 6 * 256                     # side arrays grow by at most one alignment unit each
        # N = 32 nz -> 33 nz crosses a 32-element boundary: every array grows by 32
        assert block <= b33 - b32 <= block + side
        # 33 nz -> 34 nz stays inside it (N = 66 -> 68 for D3Q19 still rounds to 96)
        assert b34 - b33 <= side
    # the padding switches on at 2^16 sites
    below = _pop_bytes(9, 65535, 1, 1, 8)
    at = _pop_bytes(9, 65536, 1, 1, 8)
    assert at - below >= 2 * 2 * 9 * 2080 * 8
    # largest lattice whose padded arrays keep 32-bit byte offsets
    from paper_1112_5547_amd import _abi
    L = _lib()
    for n, ok in ((2 ** 29 - 2112, True), (2 ** 29 - 2111, False)):
        p = _abi.Params()
        rc = L.lbm_sc_params_default(ctypes.byref(p), 9, n, 1, 1, 1.0, 1.0, 1.0)
        assert (rc == 0) == ok, n
        assert (L.lbm_sc_bytes_needed(ctypes.byref(p)) > 0) == ok


def _layout_bytes(q, nx, ny, nz, es, px):
    """The handle's bytes for population rows of px elements (the layout of
    the runtime written out: 2 buffers of 2Q arrays of NS elements, then the
    psi, rho, u, partials and totals regions, each 256-byte aligned)."""
    al = lambda b: (b + 255) // 256 * 256
    n = nx * ny * nz
    ns = (px * ny * nz + 31) // 32 * 32 + (2080 if n >= 2 ** 16 else 0)
    blocks = (n + 255) // 256
    return (2 * al(2 * q * ns * es) + al(2 * n * es) + al(2 * n * 8) + al(3 * n * 8)
            + al(blocks * 16 * 8) + al(16 * 8))


def test_population_rows_are_padded_to_32_elements():
    """From 2^16 sites on, population rows are px = nx rounded up to 32
    elements (every row starts on a cache line); smaller lattices, rows that
    are already a multiple of 32, and lattices whose padded arrays would
    leave 32-bit byte offsets keep px = nx."""
    cases = [  # (q, nx, ny, nz, es, px)
        (9, 100, 70, 1, 8, 100),          # 7,000 sites
        (9, 300, 230, 1, 4, 320),
        (19, 250, 250, 250, 4, 256),
        (19, 45, 40, 37, 8, 64),
        (19, 64, 40, 30, 8, 64),
        (19, 33, 4000, 4000, 4, 33),      # padded rows would pass 2^32 bytes per array
    ]
    for q, nx, ny, nz, es, px in cases:
        assert _pop_bytes(q, nx, ny, nz, es) == _layout_bytes(q, nx, ny, nz, es, px), (nx, ny, nz)


def test_tile_tables_and_strerror():
    L = _lib()
    for q in (9, 19):
        k = L.lbm_sc_tile_count(q)
        assert k >= 4
        for i in range(k):
            x, y = ctypes.c_int(), ctypes.c_int()
            assert L.lbm_sc_tile_get(q, i, ctypes.byref(x), ctypes.byref(y)) == 0
            if q == 9:
                assert y.value == 1
            # one ring of halo sites must fit in a block
            ring = 2 * (x.value + 2) + 2 * y.value if q == 19 else 2
            assert ring <= x.value * y.value
    assert L.lbm_sc_tile_count(5) == 0
    for st in range(-7, 1):
        assert L.lbm_sc_strerror(st)
    assert L.lbm_sc_destroy(None) == 0


def test_null_handles_are_rejected():
    L = _lib()
    assert L.lbm_sc_step(None, 1) == -1
    assert L.lbm_sc_init(None, None, None, None) == -1
    assert L.lbm_batch_run(None, 1, 0) == -1
