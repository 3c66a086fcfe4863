"""Sweep stopping rule and the two truncation-free extrapolations (host-side,
no GPU): exact recovery of polynomial data and the rule on constructed
energy sequences."""
import numpy as np
import pytest

from paper_2603_28648_amd.extrapolate import (extrapolate_inverse_bond, extrapolate_truncation,
                                              sweep_converged)


def test_sweep_rule_needs_three_agreeing_sweeps():
    assert not sweep_converged([-1.0, -1.0])
    assert sweep_converged([-1.0, -1.0 - 4e-6, -1.0 - 8e-6])
    # the older difference counts as well as the newest one
    assert not sweep_converged([-1.0, -1.0 - 2e-5, -1.0 - 2e-5])
    assert not sweep_converged([-1.0, -1.0, -1.0 - 1.1e-5])
    assert sweep_converged([-0.5, -1.0, -1.0 - 9e-6, -1.0 - 9.5e-6])
    assert not sweep_converged([-1.0, -1.0, -1.0 - 2e-7], tol=1e-7)


def test_inverse_bond_extrapolation_recovers_quadratic():
    D = np.array([256, 384, 512, 768, 1024])
    E = -30.0 + 5.0 / D - 700.0 / D ** 2
    e_ext, coef = extrapolate_inverse_bond(D, E)
    assert abs(e_ext + 30.0) < 1e-10
    assert np.allclose(coef, [-30.0, 5.0, -700.0], rtol=1e-6)


def test_truncation_extrapolation_recovers_quadratic_and_line():
    eps = np.array([3e-4, 1.5e-4, 8e-5, 3e-5])
    E = -12.0 + 40.0 * eps + 1e3 * eps ** 2
    e_ext, _ = extrapolate_truncation(eps, E)
    assert abs(e_ext + 12.0) < 1e-10
    e1, c1 = extrapolate_truncation(eps, -12.0 + 40.0 * eps, order=1)
    assert abs(e1 + 12.0) < 1e-12 and abs(c1[1] - 40.0) < 1e-8


def test_extrapolation_needs_enough_points():
    with pytest.raises(ValueError):
        extrapolate_inverse_bond([100, 200], [-1.0, -1.1])
