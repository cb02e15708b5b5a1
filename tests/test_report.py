"""The PSNR report against closed forms: a constant offset d gives 20 log10(MAX/d), the
peak is taken over all steps of the reference, identical steps give +inf, the control
line equals the PSNR of the reference plus the noise, and mismatched runs are refused."""
import numpy as np
import pytest

from paper_2409_13036_amd import report


def test_constant_offset_closed_form():
    rng = np.random.default_rng(0)
    ref = [37 + 10 * rng.random(50) for _ in range(4)]
    peak = max(a.max() for a in ref)
    # dyadic offsets: a + d is exact for these magnitudes, so the MSE is exactly d^2
    for d in (2.0 ** -17, 2.0 ** -40, 0.25):
        p = report.psnr(ref, [a + d for a in ref])
        assert np.allclose(p, 20 * np.log10(peak / d), rtol=0, atol=1e-6)
        assert abs(report.control_psnr(ref, d) - 20 * np.log10(peak / d)) < 1e-12


def test_peak_over_all_steps_and_per_step_mse():
    ref = [np.array([1.0, 2.0]), np.array([3.0, 8.0])]     # MAX(A) = 8 (second step)
    oth = [np.array([1.0, 2.5]), np.array([3.0, 8.0 - 2.0])]
    p = report.psnr(ref, oth)
    assert np.isclose(p[0], 20 * np.log10(8 / np.sqrt(0.125)))   # MSE = 0.25 / 2
    assert np.isclose(p[1], 20 * np.log10(8 / np.sqrt(2.0)))     # MSE = 4 / 2


def test_identical_steps_and_errors():
    ref = [np.ones(3), 2 * np.ones(3)]
    assert np.all(np.isinf(report.psnr(ref, [a.copy() for a in ref])))
    with pytest.raises(ValueError):
        report.psnr(ref, ref[:1])
    with pytest.raises(ValueError):
        report.psnr(ref, [np.ones(3), np.ones(4)])
    s = report.summary(ref, [a + 1e-6 for a in ref])
    assert s["steps"] == 2 and set(s["control_db"]) == {"1e-05", "1e-12"}
