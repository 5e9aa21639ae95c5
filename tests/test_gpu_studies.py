"""FP32 shifted against FP64 at the statistical level (spinodal domain growth)
and the 128^3 static drop's measured quantities; the host-side structure
factor is pinned against a closed form first."""
import numpy as np
import pytest

from gpu_common import say


def test_domain_length_of_a_single_mode():
    """phi = cos(2 pi m x / L): S(k) has weight only at |k| = 2 pi m / L, so l = L / m."""
    from paper_1112_5547_amd.studies import domain_length
    L, m = 64, 4
    x = np.arange(L)
    phi = np.broadcast_to(np.cos(2 * np.pi * m * x / L), (L, L, L)).copy()
    assert abs(domain_length(phi) - L / m) < 1e-9


@pytest.mark.gpu
def test_spinodal_fp32_shifted_tracks_fp64_statistically():
    from paper_1112_5547_amd.studies import spinodal_study
    say("spinodal study 96^3, 1200 steps, fp64 and fp32_shifted")
    r = spinodal_study(L=96, steps=1200, every=300)
    a, b = r["fp64"], r["fp32_shifted"]
    assert a[-1]["domain_length"] > 2 * a[0]["domain_length"]      # coarsening happened
    for ra, rb in zip(a[2:], b[2:]):
        assert abs(rb["domain_length"] - ra["domain_length"]) <= 0.02 * ra["domain_length"]
    for row in a:
        assert abs(row["mass_drift_A"]) <= 1200 * 2.0 ** -52 * 8
        assert row["n_nonfinite"] == 0
    for row in b:
        assert abs(row["mass_drift_A"]) <= 1e-5


@pytest.mark.gpu
def test_drop_128cube_fp32_against_fp64():
    """128^3 D3Q19 drop (R = 24, tau = 1, G = 1.3, seed 2), 1000 steps."""
    from paper_1112_5547_amd.studies import compare_drop, drop_study
    say("drop study 128^3, 1000 steps, fp64 and fp32_shifted")
    c = compare_drop(drop_study(L=128, steps=1000))
    assert c["dp_fp64"] > 0
    assert c["dp_rel"] <= 0.01
    assert c["max_u_rel"] <= 0.01
    assert c["max_abs_rho_A"] <= 1e-4
    assert abs(c["mass_drift_A_fp64"]) <= 1000 * 2.0 ** -52 * 8
    assert abs(c["R_eff_fp32"] - c["R_eff_fp64"]) <= 0.01 * c["R_eff_fp64"]


@pytest.mark.gpu
def test_spinodal_256cube_5000_steps_precision():
    """The precision configuration: D3Q19 256^3 spinodal (G = 1.6, tau = 1,
    seed 3), 5000 steps in FP64 and in FP32 shifted storage, compared at the
    statistical level.  Bounds: domain lengths within 2 %; FP64 mass drift
    within 8 roundings per step and |sum j| <= 1e-8; FP32 mass drift <= 2e-5
    relative and the lattice momentum |sum j| <= 1e-9 N steps, i.e. an
    average momentum bias under 1e-9 per site and step, about a hundredth of
    an FP32 unit in the last place of the stored populations (|h| ~ 0.1)."""
    from paper_1112_5547_amd.studies import spinodal_study
    L, steps = 256, 5000
    say("spinodal study 256^3, 5000 steps, fp64 and fp32_shifted")
    r = spinodal_study(L=L, steps=steps, every=2500)
    a, b = r["fp64"], r["fp32_shifted"]
    say(f"domain lengths fp64 {[round(x['domain_length'], 3) for x in a]} "
        f"fp32 {[round(x['domain_length'], 3) for x in b]}; momentum fp64 {a[-1]['mom']:.3e} "
        f"fp32 {b[-1]['mom']:.3e}; mass drift fp64 {a[-1]['mass_drift_A']:.3e} "
        f"fp32 {b[-1]['mass_drift_A']:.3e}")
    assert a[-1]["domain_length"] > 10 * a[0]["domain_length"]      # coarsening happened
    assert abs(b[-1]["domain_length"] - a[-1]["domain_length"]) <= 0.02 * a[-1]["domain_length"]
    assert abs(a[-1]["mass_drift_A"]) <= steps * 2.0 ** -52 * 8
    assert a[-1]["mom"] <= 1e-8
    assert abs(b[-1]["mass_drift_A"]) <= 2e-5
    assert b[-1]["mom"] <= 1e-9 * L ** 3 * steps
    assert a[-1]["n_nonfinite"] == 0 and b[-1]["n_nonfinite"] == 0
