"""Seeded MP 2-B inputs (§2, §5.2): k = k1 + (k2 - k1) χ with χ a random
function onto [0, 1]; the grid puts max(k) h at 0.625."""
import numpy as np

from paper_2308_13476_amd import workloads as W


def test_profiles_span_exactly_the_unit_interval_and_k_range():
    for chi in [W.chi_smooth(80, 5), W.chi_sharp(120, 6), W.chi_smooth(33, 1), W.chi_sharp(16, 2)]:
        assert chi.min() == 0.0 and chi.max() == 1.0
        k = np.sqrt(W.k2_from_chi(chi, 10, 75))
        assert abs(k.min() - 10.0) < 1e-12 and abs(k.max() - 75.0) < 1e-12


def test_profiles_are_seeded():
    np.testing.assert_array_equal(W.chi_sharp(40, 6), W.chi_sharp(40, 6))
    np.testing.assert_array_equal(W.chi_smooth(40, 5), W.chi_smooth(40, 5))
    assert not np.array_equal(W.chi_sharp(40, 6), W.chi_sharp(40, 7))


def test_smooth_profile_changes_gradually_and_sharp_profile_does_not():
    # mean jump between horizontal neighbours relative to the full range
    def jump(chi):
        return float(np.mean(np.abs(np.diff(chi, axis=1))))
    assert jump(W.chi_smooth(120, 5)) < 0.02
    assert jump(W.chi_sharp(120, 6)) > 0.25  # independent U(0,1): mean |difference| = 1/3


def test_grid_rule_kh_0625():
    assert W.mp2b_grid(50) == 80 and W.mp2b_grid(75) == 120
    assert abs(75.0 / W.mp2b_grid(75) - 0.625) < 1e-12
