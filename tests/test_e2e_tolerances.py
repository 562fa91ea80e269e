"""The statistical bounds of the end-to-end GPU tests (host arithmetic only)."""
import numpy as np

from tests import e2e


def test_bound_is_three_sigma_for_known_uncertainties():
    assert abs(e2e.bound3([(0.3, np.inf), (0.4, np.inf)]) - 1.5) < 1e-12


def test_bound_uses_student_t_for_few_realisations():
    # four realisations: 3 degrees of freedom, t(0.99865, 3) = 9.2187
    se, dof = e2e.mean_se([1.0, 2.0, 3.0, 4.0])
    assert dof == 3 and abs(se - np.std([1, 2, 3, 4], ddof=1) / 2) < 1e-15
    assert abs(e2e.bound3([(se, dof)]) / se - 9.2187) < 1e-3


def test_welch_satterthwaite_degrees_of_freedom():
    # two equal parts of 3 degrees of freedom each: 6; a known part with
    # a sampled one: more than the sampled part's own
    s, d = e2e.combine([(1.0, 3), (1.0, 3)])
    assert abs(s - np.sqrt(2)) < 1e-15 and abs(d - 6.0) < 1e-12
    s, d = e2e.combine([(0.01, 1), (0.03, np.inf)])
    assert abs(d - 100.0) < 1e-9
    # the bound then approaches 3 sigma
    assert 3.0 * s < e2e.bound3([(0.01, 1), (0.03, np.inf)]) < 3.1 * s
