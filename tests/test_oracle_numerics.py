"""Pins of the oracle's complex and bicomplex numerics (Sec. 3).

The oracle's derivatives are checked against closed-form derivatives of the
paper's test function f(x) = (e^x + x^3 + x)/(x + 1) (the function of the
AD/FD/CSFD comparison table), the second-order convergence of the full complex
step (eq. csfd: error O(h^2)), and the symmetry of the mixed bicomplex
derivative (eq. csfd_hessian).
"""
import math

import numpy as np
import pytest

import oracle as O


def f(x):
    return (math.exp(x) + x ** 3 + x) / (x + 1)


def f1(x):
    N, N1, D = math.exp(x) + x ** 3 + x, math.exp(x) + 3 * x * x + 1, x + 1
    return N1 / D - N / D ** 2


def f2(x):
    N, N1, N2, D = math.exp(x) + x ** 3 + x, math.exp(x) + 3 * x * x + 1, math.exp(x) + 6 * x, x + 1
    return N2 / D - 2 * N1 / D ** 2 + 2 * N / D ** 3


XS = [0.0, 0.1234, 0.5, 0.77, 1.0]


@pytest.mark.parametrize("x", XS)
def test_csfd_first_derivative_matches_closed_form(x):
    h = 1e-20
    out = O.eval_f(O.seed(1, h=h), x)
    assert out[0] == pytest.approx(f(x), rel=1e-15)
    assert abs(out[1] / h - f1(x)) <= 2e-15 * abs(f1(x))


def test_csfd_error_decays_as_h_squared():
    # Im f(x + ih)/h = f'(x) - f'''(x) h^2/6 + O(h^4): slope 2 in log-log
    x = 0.5
    hs = np.array([1e-1, 3e-2, 1e-2, 3e-3, 1e-3])
    errs = np.array([abs(O.eval_f(O.seed(1, h=h), x)[1] / h - f1(x)) for h in hs])
    slopes = np.diff(np.log(errs)) / np.diff(np.log(hs))
    assert np.all(np.abs(slopes - 2.0) < 0.05), slopes


def test_csfd_step_below_sqrt_eps_is_exact():
    # "when h ~ sqrt(eps) CSFD is as accurate as the analytic derivative"
    x = 0.3
    for h in (1e-8, 1e-12, 1e-30, 1e-100):
        assert abs(O.eval_f(O.seed(1, h=h), x)[1] / h - f1(x)) <= 4e-15 * abs(f1(x))


@pytest.mark.parametrize("x", XS)
def test_bicomplex_second_derivative(x):
    h = 1e-20
    out = O.eval_f(O.seed(2, h=h), x)  # x + h i1 + h i2
    assert abs(out[1] / h - f1(x)) <= 2e-15 * abs(f1(x))
    assert abs(out[2] / h - f1(x)) <= 2e-15 * abs(f1(x))
    assert abs(out[3] / h ** 2 - f2(x)) <= 1e-13 * abs(f2(x))


def test_bicomplex_mixed_derivative_symmetric_and_matches_fd():
    x, y, h = 0.4, 0.7, 1e-20
    s = O.seed(2, h=h)
    a = O.eval_g(s, x, y, 1, 2)[3] / h ** 2   # x on i1, y on i2
    b = O.eval_g(s, x, y, 2, 1)[3] / h ** 2   # y on i1, x on i2
    assert abs(a - b) <= 1e-13 * abs(a)
    # central difference (in y) of the CSFD first derivative in x
    c = O.seed(1, h=h)
    d = 1e-5
    gp = O.eval_g(c, x, y + d, 1, 0)[1] / h
    gm = O.eval_g(c, x, y - d, 1, 0)[1] / h
    assert abs((gp - gm) / (2 * d) - a) <= 1e-8 * abs(a)


def test_real_run_has_no_imaginary_parts():
    assert O.eval_f(O.seed(0), 0.3).shape == (1,)
    assert O.eval_f(O.seed(0), 0.3)[0] == pytest.approx(f(0.3), rel=1e-15)
