"""Pins of the oracle's complex SE(3) exponential (Sec. 4.1, eqs. lie,
rotvector, rotation_jacobi) against scipy's matrix exponential of the twist
matrix (a Pade approximant, independent of the Rodrigues series used here),
evaluated in complex arithmetic for the derivative, and against the Lie
generators and the structure of SO(3)."""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle as O

H = 1e-20


def twist(xi):
    phi, rho = xi[:3], xi[3:]
    M = np.zeros((4, 4), dtype=np.result_type(xi))
    M[0, 1], M[0, 2], M[1, 0], M[1, 2], M[2, 0], M[2, 1] = -phi[2], phi[1], phi[2], -phi[0], -phi[1], phi[0]
    M[:3, 3] = rho
    return M


def xis():
    rng = np.random.default_rng(7)
    out = [np.zeros(6), np.array([1e-9, -2e-9, 3e-9, 0.1, 0.2, -0.3])]
    for scale in (1e-4, 1e-2, 0.0999, 0.1001, 0.5, 2.0, 3.0):
        v = rng.standard_normal(6)
        v[:3] *= scale / np.linalg.norm(v[:3])
        out.append(v)
    return out


@pytest.mark.parametrize("xi", xis())
def test_real_exp_matches_expm(xi):
    T = O.se3_exp(O.seed(0), xi)[..., 0]
    assert np.allclose(T, expm(twist(xi)), rtol=0, atol=2e-15 * max(1.0, np.abs(xi).max()))


@pytest.mark.parametrize("xi", xis())
@pytest.mark.parametrize("d", range(6))
def test_complex_step_derivative_matches_complex_expm(xi, d):
    s = O.seed(1, h=H)
    x = O.lift(xi, s)
    x[d, 1] = H
    T = O.se3_exp(s, x)
    z = xi.astype(np.complex128)
    z[d] += 1j * H
    ref = expm(twist(z))
    assert np.allclose(T[..., 0], ref.real, rtol=0, atol=2e-15 * max(1.0, np.abs(xi).max()))
    dref = ref.imag / H
    assert np.allclose(T[..., 1] / H, dref, rtol=0, atol=1e-13 * max(1.0, np.abs(dref).max()))


def test_generators_at_zero():
    s = O.seed(1, h=H)
    for d in range(6):
        x = O.lift(np.zeros(6), s)
        x[d, 1] = H
        G = O.se3_exp(s, x)[..., 1] / H
        e = np.zeros(6)
        e[d] = 1.0
        assert np.array_equal(G, twist(e))


@pytest.mark.parametrize("xi", xis())
def test_rotation_structure(xi):
    s = O.seed(1, h=H)
    x = O.lift(xi, s)
    x[0, 1] = H
    T = O.se3_exp(s, x)
    R, dR = T[:3, :3, 0], T[:3, :3, 1] / H
    assert np.allclose(R.T @ R, np.eye(3), atol=1e-14)
    S = R.T @ dR                      # tangent of SO(3) at R is R * skew
    assert np.allclose(S, -S.T, atol=1e-13)


def test_series_and_closed_form_agree_at_threshold():
    # re(theta^2) = 1e-2 switches from the even series to sin/cos
    base = np.array([0.06, -0.07, 0.0, 0.3, -0.2, 0.1])
    base[2] = np.sqrt(1e-2 - base[0] ** 2 - base[1] ** 2)
    lo = O.se3_exp(O.seed(0), base * (1 - 1e-9))[..., 0]
    hi = O.se3_exp(O.seed(0), base * (1 + 1e-9))[..., 0]
    assert np.abs(lo - hi).max() < 1e-9


def test_bicomplex_second_derivative_symmetric():
    s = O.seed(2, h=H)
    xi = np.array([0.2, -0.1, 0.3, 0.5, 0.1, -0.2])
    x = O.lift(xi, s)
    x[0, 1] = H   # phi_x on i1
    x[4, 2] = H   # rho_y on i2
    a = O.se3_exp(s, x)[..., 3] / H ** 2
    y = O.lift(xi, s)
    y[4, 1] = H
    y[0, 2] = H
    b = O.se3_exp(s, y)[..., 3] / H ** 2
    assert np.allclose(a, b, atol=1e-14)
    # against central differences of the complex-step first derivative
    c = O.seed(1, h=H)
    dd = 1e-6
    def first(v):
        z = O.lift(v, c)
        z[0, 1] = H
        return O.se3_exp(c, z)[..., 1] / H
    ep = xi.copy(); ep[4] += dd
    em = xi.copy(); em[4] -= dd
    fd = (first(ep) - first(em)) / (2 * dd)
    assert np.allclose(a, fd, atol=1e-8)
