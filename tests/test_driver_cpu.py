"""Host-side schedules of the placement loop (Section IV-A formulas)."""
import math

import pytest

from paper_1312_4587_amd.driver import (gamma_of_tau, mu_of_hpwl_change, nesterov_beta,
                                        step_length)


def test_gamma_schedule_values():
    # 8 w_b 10^(20/9 (tau - 0.1) - 1): 0.8 w_b at tau = 0.1, 80 w_b at tau = 1
    assert gamma_of_tau(0.1, 2.0) == pytest.approx(1.6, rel=1e-14)
    assert gamma_of_tau(1.0, 1.0) == pytest.approx(80.0, rel=1e-14)
    assert gamma_of_tau(0.55, 1.0) == pytest.approx(8.0, rel=1e-14)
    assert gamma_of_tau(0.3, 1.0) < gamma_of_tau(0.4, 1.0)


def test_lambda_scaling_is_bounded():
    assert mu_of_hpwl_change(0.0) == pytest.approx(1.1)
    assert mu_of_hpwl_change(3.5e5) == pytest.approx(1.0)
    assert mu_of_hpwl_change(1e9) == 0.75
    assert mu_of_hpwl_change(-1e9) == 1.1
    assert mu_of_hpwl_change(7e5) == pytest.approx(1.1 ** -1.0)


def test_nesterov_sequence():
    a, beta = nesterov_beta(1.0)
    assert beta == 0.0 and a == pytest.approx((1 + math.sqrt(5)) / 2)
    for _ in range(200):
        a, beta = nesterov_beta(a)
        assert 0.0 <= beta < 1.0
    assert beta > 0.98


def test_step_length_bounds():
    assert step_length(1.0, 4.0, 3.0, 0.01, 10.0, first=True) == 10.0
    assert step_length(1.0, 4.0, 3.0, 0.01, 10.0, first=False) == pytest.approx(1.5)
    assert step_length(1.0, 4.0, 3.0, 0.01, 1.0, first=False) == 1.0
    assert step_length(1e-8, 4.0, 3.0, 0.01, 1.0, first=False) == 0.01
    assert step_length(1.0, 0.0, 3.0, 0.01, 1.0, first=False) == 1.0
