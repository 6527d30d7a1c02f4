"""Pins of the oracle's constant-velocity estimate and of its state-loaded
frame step.

Constant velocity (the ICP start when the configuration asks for it; the
paper itself starts from the previous pose, Sec. 4.1 after eq. icp):

* on a constant-twist trajectory T_k = exp(k xi) T_0 the estimate
  T_1 T_2^-1 T_1 is exactly the next pose exp((k+1) xi) T_0 (a group
  identity), checked against scipy's matrix exponential;
* the polar Newton steps return a rotation whose R^T R is the identity to
  rounding, from inputs that are off orthonormal by 1e-6, and leave an exact
  rotation unchanged to rounding;
* when either frame was lost the estimate is the previous pose, bit for bit;
* its complex-step tangent equals central differences of the real estimate.

State-loaded frame steps: chaining ``frame_step`` from an empty state
reproduces ``run_sequence`` bit for bit (poses, per-frame counters, volume),
with and without constant velocity; the raycast footprint only observes.
"""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle as O
from test_oracle_sequence import small_cfg, small_seq, twist


def _pose(xi, T0):
    return expm(twist(np.asarray(xi, float))) @ T0


def _T0():
    rng = np.random.default_rng(3)
    return _pose(rng.normal(size=6) * 0.4, np.eye(4))


def test_constant_twist_extrapolates_exactly():
    xi = np.array([0.010, -0.020, 0.015, 0.030, 0.010, -0.020])
    T0 = _T0()
    s = O.seed(0)
    for k in (1, 5, 20):
        T1, T2, T3 = _pose(k * xi, T0), _pose((k - 1) * xi, T0), _pose((k + 1) * xi, T0)
        P = O.const_vel(s, O.lift(T1, s), O.lift(T2, s))[..., 0]
        assert np.abs(P - T3).max() <= 1e-14 * max(1.0, np.abs(T3).max())


def test_polar_steps_reorthonormalise():
    rng = np.random.default_rng(7)
    T0 = _T0()
    s = O.seed(0)
    for trial in range(5):
        T1 = _pose(rng.normal(size=6) * 0.05, T0)
        T2 = _pose(rng.normal(size=6) * 0.05, T0)
        # departure from orthonormality of order 1e-6 in both inputs
        T1[:3, :3] += 1e-6 * rng.normal(size=(3, 3))
        T2[:3, :3] += 1e-6 * rng.normal(size=(3, 3))
        P = O.const_vel(s, O.lift(T1, s), O.lift(T2, s))[..., 0]
        R = P[:3, :3]
        assert np.abs(R.T @ R - np.eye(3)).max() <= 1e-15
        assert np.linalg.det(R) > 0
        # without the steps the product is ~3e-6 off orthonormal
        R_raw = (T1 @ np.linalg.inv(T2) @ T1)[:3, :3]
        assert np.abs(R_raw.T @ R_raw - np.eye(3)).max() > 1e-7


def test_exact_rotation_unchanged():
    T0 = _T0()
    s = O.seed(0)
    xi = np.array([0.2, -0.1, 0.3, 0.1, 0.2, 0.3])
    T1, T2 = _pose(2 * xi, T0), _pose(xi, T0)
    P = O.const_vel(s, O.lift(T1, s), O.lift(T2, s))[..., 0]
    Q = T1 @ np.linalg.inv(T2) @ T1
    assert np.abs(P - Q).max() <= 1e-14


def test_lost_frame_keeps_previous_pose():
    T0 = _T0()
    s = O.seed(1, O.P_TRUNC)
    T1 = O.lift(_pose([0.1, 0, 0, 0.2, 0, 0], T0), s)
    T1[..., 1] = np.random.default_rng(0).normal(size=(4, 4)) * 1e-20
    T2 = O.lift(T0, s)
    assert np.array_equal(O.const_vel(s, T1, T2, both_tracked=False), T1)


def test_complex_tangent_matches_central_differences():
    T0 = _T0()
    xi1 = np.array([0.02, 0.01, -0.03, 0.05, 0.02, 0.01])
    xi2 = np.array([0.01, 0.00, -0.01, 0.02, 0.01, 0.00])
    e = np.array([0.3, -0.2, 0.5, 1.0, -0.4, 0.7])   # direction in the twist of T1
    h = 1e-20
    s = O.seed(1, O.P_TRUNC, h=h)
    # T1(t) = exp(xi1 + t e) T0 with a complex t: lift through the oracle's own exp
    xi_c = np.zeros((6, 2))
    xi_c[:, 0] = xi1
    xi_c[:, 1] = h * e
    T1c = O.se3_exp(s, xi_c)
    T1c = np.einsum("ijc,jk->ikc", T1c, T0)
    T2 = O.lift(_pose(xi2, T0), s)
    P = O.const_vel(s, T1c, T2)
    g = P[..., 1] / h
    s0 = O.seed(0)
    best = np.inf
    for d in (1e-4, 1e-5, 1e-6):
        Pp = O.const_vel(s0, O.lift(_pose(xi1 + d * e, T0), s0), O.lift(_pose(xi2, T0), s0))[..., 0]
        Pm = O.const_vel(s0, O.lift(_pose(xi1 - d * e, T0), s0), O.lift(_pose(xi2, T0), s0))[..., 0]
        fd = (Pp - Pm) / (2 * d)
        best = min(best, np.abs(fd - g).max() / np.abs(g).max())
    assert best <= 1e-8


def _chain(c, s, depths, T0):
    st = O.State(c, s)
    T0l = O.lift(T0, s)
    st.T1 = T0l.copy()
    st.T2 = T0l.copy()
    poses, stats = [], []
    for k in range(depths.shape[0]):
        stats.append(O.frame_step(c, s, st, depths[k]))
        poses.append(st.T1.copy())
    return np.array(poses), np.array(stats), st


@pytest.mark.parametrize("init", [0, 1])
def test_state_loaded_steps_reproduce_the_sequence(init):
    depths, T0, _ = small_seq()
    c = small_cfg(init=init)
    s = O.seed(1, O.P_TRUNC, h=1e-20)
    ref = O.run_sequence(c, s, depths, T0, want_volume=True)
    poses, stats, st = _chain(c, s, depths, T0)
    assert np.array_equal(poses, ref["poses"])
    assert np.array_equal(stats, ref["stats"])
    assert np.array_equal(st.F, ref["F"]) and np.array_equal(st.W, ref["W"])


def test_footprint_only_observes():
    depths, T0, _ = small_seq()
    c = small_cfg()
    s = O.seed(1, O.P_TRUNC, h=1e-20)
    st = O.State(c, s)
    st.T1 = O.lift(T0, s)
    st.T2 = st.T1.copy()
    O.frame_step(c, s, st, depths[0])
    touch, hits = O.raycast_footprint(c, s, st.F, st.W, st.T1)
    assert hits == int(st.valid.sum())
    # every voxel marked is inside the volume's cells; hits touch a subset of the
    # marched cells' neighbourhood, and unobserved voxels are touched too (the
    # march reads a cell before knowing all its corners are observed)
    n1 = int(np.count_nonzero(touch & 1))
    n2 = int(np.count_nonzero(touch & 2))
    assert n1 > 0 and n2 > 0
    assert n2 < n1
    # a second footprint of the same state is the same set
    touch2, _ = O.raycast_footprint(c, s, st.F, st.W, st.T1)
    assert np.array_equal(touch, touch2)


def test_constant_velocity_sequence_differs_only_from_frame_two():
    depths, T0, _ = small_seq()
    s = O.seed(0)
    a = O.run_sequence(small_cfg(init=0), s, depths, T0)
    b = O.run_sequence(small_cfg(init=1), s, depths, T0)
    assert np.array_equal(a["poses"][:2], b["poses"][:2])
    # tracking converges to nearly the same poses from either start
    assert np.abs(a["poses"][2:] - b["poses"][2:]).max() < 1e-3
