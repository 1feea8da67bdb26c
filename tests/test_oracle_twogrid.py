"""Weak pin of the two-grid analysis against the paper's Table 1 (§4).

The Bézier + CSL column is reproduced within 0.02. The other columns only keep
the paper's ordering; their printed values are not reproduced under the
readings used here (parity unpinned for those three columns).
"""
import json
import os

import pytest

from oracle.twogrid import spectral_norm, spectral_radius, two_grid_matrix

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
G = json.load(open(os.path.join(GOLDEN, "table1_two_grid_norms.json")))


@pytest.mark.parametrize("idx", [0, 1, 2, 3])
def test_bezier_csl_norm_matches_table1(idx):
    k, n = G["k"][idx], G["n"][idx]
    T = two_grid_matrix(k, n, beta2=0.7, transfer="bezier", coarse_on="C")
    assert abs(spectral_norm(T) - G["bezier_C"][idx]) < 0.02
    assert spectral_radius(T) < 1.0


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_ordering_of_table1_columns(idx):
    k, n = G["k"][idx], G["n"][idx]
    norms = {(t, c): spectral_norm(two_grid_matrix(k, n, 0.7, t, c)) for t in ["linear", "bezier"] for c in "AC"}
    assert norms[("bezier", "C")] < 1.0
    assert norms[("bezier", "A")] > norms[("bezier", "C")]
    assert norms[("linear", "A")] > norms[("linear", "C")] > 1.0
    if k >= 10:
        assert norms[("bezier", "A")] > 1.0
