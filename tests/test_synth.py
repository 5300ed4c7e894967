"""Seeded input generators (synth/): the per-member friction of the
ensemble runs on planar and triangle faults."""
import numpy as np

from synth import (config_fault, config_triangle_fault, ensemble_params, planar_rect_fault,
                   triangle_friction_params)


def test_ensemble_params_ranges_and_sigma():
    tri = config_triangle_fault("thrust_16x12")
    p = ensemble_params(tri, 5, 3)
    n = tri.n
    assert p["a"].shape == p["b"].shape == p["dc"].shape == (n, 5)
    amb = p["a"] - p["b"]
    assert np.all(p["b"] == 0.015) and amb.min() >= -0.006 and amb.max() < 0.004
    assert p["dc"].min() >= 0.005 and p["dc"].max() <= 0.05
    # sigma: the depth profile of the triangle fault, shared by every member
    np.testing.assert_array_equal(p["sigma"], triangle_friction_params(tri)["sigma"])
    assert p["sigma"].min() == 20.0e6 and p["sigma"].max() == 120.0e6
    # a planar fault keeps 50 MPa; the draws depend only on (n, members, seed)
    flat = planar_rect_fault(tri.n, 1, 100.0, 30.0, "dip")
    q = ensemble_params(flat, 5, 3)
    assert np.all(q["sigma"] == 50.0e6)
    np.testing.assert_array_equal(q["a"], p["a"])
    np.testing.assert_array_equal(q["dc"], p["dc"])
    # members differ, seeds differ
    assert not np.array_equal(p["a"][:, 0], p["a"][:, 1])
    assert not np.array_equal(ensemble_params(config_fault("dip30_48x24"), 5, 4)["a"],
                              ensemble_params(config_fault("dip30_48x24"), 5, 3)["a"])
