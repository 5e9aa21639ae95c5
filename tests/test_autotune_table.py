"""Lookup rules of the tuned-configuration table (host logic, no device):
exact key first, then the nearest tuned size of the same lattice type,
precision and forcing scheme; a Guo lattice with no Guo entries of its type
falls back to the velocity-shift entries of its precision."""
from paper_1112_5547_amd import autotune

TABLE = {
    "19:256:256:256:fp64": {"variant": 0, "tx": 64, "ty": 8, "mb": 128},
    "19:128:128:128:fp64": {"variant": 0, "tx": 64, "ty": 8, "mb": 16},
    "19:256:256:256:fp64+guo": {"variant": 3, "tx": 32, "ty": 8, "mb": 64},
    "9:512:512:1:fp32_shifted": {"variant": 2, "tx": 256, "ty": 1, "mb": 4},
}


def test_exact_and_nearest_keys():
    assert autotune.lookup(19, 256, 256, 256, "fp64", TABLE) == (0, 64, 8, 128)
    assert autotune.lookup(19, 120, 120, 120, "fp64", TABLE) == (0, 64, 8, 16)
    assert autotune.lookup(19, 96, 96, 8, "fp64", TABLE) == (0, 64, 8, 8)   # mb clipped to nz
    assert autotune.lookup(9, 64, 64, 1, "fp64", TABLE) is None             # nothing of the type


def test_guo_entries_are_separate_and_fall_back_to_the_shift():
    assert autotune.lookup(19, 256, 256, 256, "fp64", TABLE, "guo") == (3, 32, 8, 64)
    assert autotune.lookup(19, 200, 200, 200, "fp64", TABLE, "guo") == (3, 32, 8, 64)
    # no Guo entry for D2Q9 FP32: the velocity-shift choice of that precision
    assert autotune.lookup(9, 500, 500, 1, "fp32_shifted", TABLE, "guo") == (2, 256, 1, 4)
    assert autotune._key(19, 8, 8, 8, "fp64", "guo") == "19:8:8:8:fp64+guo"
