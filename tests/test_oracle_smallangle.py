"""Pins of the oracle's original-KinectFusion update form (eq. icp_approx:
the increment's rotation taken as I + [phi]x, cos ~ 1 and sin ~ angle; then
two polar Newton steps keep the pose rigid), the comparison form of the
paper's exact-exponential update.

* it agrees with the exact exponential to first order: the difference
  shrinks 4x when the increment halves, and the complex-step derivative at
  zero is the same Lie generator;
* the polar decomposition of I + [phi]x is the rotation by atan|phi| about
  phi (a closed form): the re-orthonormalised increment equals it;
* a tracked sequence with this form runs, and differs from the exact form.
"""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle as O
from test_oracle_sequence import small_cfg, small_seq, twist


def _rot(axis_angle):
    return expm(twist(np.concatenate([axis_angle, np.zeros(3)])))[:3, :3]


def test_first_order_agreement_with_the_exponential():
    s = O.seed(0)
    xi0 = np.array([0.02, -0.015, 0.01, 0.03, -0.02, 0.01])
    errs = []
    for k in range(4):
        xi = xi0 / 2 ** k
        sa = O.small_angle_update(s, O.lift(xi, s), O.lift(np.eye(4), s))[..., 0]
        ex = expm(twist(xi))
        errs.append(np.abs(sa - ex).max())
    ratios = [errs[k] / errs[k + 1] for k in range(3)]
    assert all(3.5 < r < 4.5 for r in ratios), ratios


@pytest.mark.parametrize("d", range(6))
def test_derivative_at_zero_is_the_generator(d):
    h = 1e-20
    s = O.seed(1, d, h=h)
    xi = np.zeros((6, 2))
    xi[d, 1] = h
    T = O.small_angle_update(s, xi, O.lift(np.eye(4), s))
    e = np.zeros(6)
    e[d] = 1.0
    assert np.abs(T[..., 1] / h - twist(e)).max() < 1e-14
    assert np.abs(T[..., 0] - np.eye(4)).max() == 0.0


def test_polar_of_small_angle_is_rotation_by_atan():
    s = O.seed(0)
    rng = np.random.default_rng(4)
    T0 = expm(twist(rng.normal(size=6) * 0.3))
    for theta in (1e-3, 5e-3, 2e-2):
        ax = rng.normal(size=3)
        ax /= np.linalg.norm(ax)
        xi = np.concatenate([theta * ax, rng.normal(size=3) * 0.02])
        out = O.small_angle_update(s, O.lift(xi, s), O.lift(T0, s))[..., 0]
        R_ref = _rot(np.arctan(theta) * ax) @ T0[:3, :3]
        assert np.abs(out[:3, :3] - R_ref).max() < 1e-10, theta
        # translation: (I + [phi]x) t0 + rho
        K = twist(np.concatenate([xi[:3], np.zeros(3)]))[:3, :3]
        assert np.abs(out[:3, 3] - ((np.eye(3) + K) @ T0[:3, 3] + xi[3:])).max() < 1e-15


def test_sequence_with_small_angle_form_tracks_and_differs():
    depths, T0, gt = small_seq()
    s = O.seed(0)
    a = O.run_sequence(small_cfg(update=0), s, depths, T0)
    b = O.run_sequence(small_cfg(update=1), s, depths, T0)
    assert a["stats"][:, 0].sum() == 0 and b["stats"][:, 0].sum() == 0
    assert not np.array_equal(a["poses"][1:], b["poses"][1:])
    for P in b["poses"][..., 0]:
        R = P[:3, :3]
        assert np.abs(R.T @ R - np.eye(3)).max() < 1e-12
    # both converge to nearly the same poses at this small motion
    assert np.abs(a["poses"] - b["poses"]).max() < 1e-3
