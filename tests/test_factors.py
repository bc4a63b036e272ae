"""Host logic of the convergence-factor experiment: the averaged factor of a
residual history (no GPU)."""
import math

import numpy as np

from paper_1907_12334_amd.factors import averaged_factors, expected_factor


def test_geometric_history_gives_its_ratio():
    k = np.arange(21)
    r = np.stack([0.3 ** k, 0.05 ** k])
    f = averaged_factors(r, floor=1e-30)
    assert np.allclose(f, [0.3, 0.05], rtol=1e-12)


def test_floor_cuts_the_rounding_plateau():
    k = np.arange(31)
    row = np.maximum(0.1 ** k, 1e-14)        # reaches the plateau after 14 cycles
    f = averaged_factors(row[None, :], floor=1e-10)
    assert math.isclose(f[0], 0.1, rel_tol=1e-12)   # last cycle above the floor is k = 10


def test_divergence_and_non_finite_are_not_converged():
    r = np.array([[1.0, 0.9, 1.3], [1.0, np.nan, 0.1], [1.0, 0.5, 0.25]])
    f = averaged_factors(r)
    assert f[0] == math.inf and f[1] == math.inf and math.isclose(f[2], 0.5)
    assert expected_factor(r) is None
    assert math.isclose(expected_factor(r[2:]), 0.5)


def test_exact_first_cycle():
    r = np.array([[1.0, 1e-16, 1e-17]])
    assert averaged_factors(r)[0] == 1e-16
