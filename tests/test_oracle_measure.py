"""Pins of the oracle's surface measurement (Sec. 4.1: bilateral filter, depth
promotion eq. csfd_depth and its derivatives eq. pvnpd, pyramid, eqs. vertex and
normal) on depth maps with closed-form answers: constant and planar depth,
linear ramps and step edges."""
import numpy as np
import pytest

import oracle as O

W, H = 40, 30
FX, FY, CX, CY = 35.0, 36.0, 19.5, 14.5


def cfg(**kw):
    d = dict(width=W, height=H, fx=FX, fy=FY, cx=CX, cy=CY)
    d.update(kw)
    return O.config(None, **d)


def plane_depth(n, d):
    """Depth of the plane n . X = d seen from the origin (camera frame)."""
    x = (np.arange(W) - CX) / FX
    y = (np.arange(H) - CY) / FY
    ray = np.stack(np.broadcast_arrays(x[None, :], y[:, None], np.ones((1, 1))), -1)
    return d / (ray @ n), ray


def test_constant_depth_is_a_fixed_point_and_uniform_shift_has_unit_derivative():
    D = np.full((H, W), 1.7)
    s = O.seed(1, O.P_DEPTH, h=1e-20)
    out = O.measure(cfg(), s, D, np.ones((H, W)))
    for lvl in out:
        v = lvl["D"]
        assert np.allclose(v[..., 0], 1.7, rtol=0, atol=1e-15)
        assert np.allclose(v[..., 1] / 1e-20, 1.0, rtol=0, atol=1e-14)


def test_bilateral_preserves_a_step_edge():
    D = np.full((H, W), 1.0)
    D[:, W // 2:] = 2.0
    out = O.measure(cfg(), O.seed(0), D)[0]["D"][..., 0]
    assert np.abs(out[:, : W // 2] - 1.0).max() < 1e-12
    assert np.abs(out[:, W // 2:] - 2.0).max() < 1e-12


def test_pyramid_of_a_linear_ramp_samples_the_centre():
    # symmetric binomial weights reproduce a linear function at the centre tap
    D = 1.0 + 0.001 * np.arange(W)[None, :] + 0.002 * np.arange(H)[:, None]
    out = O.measure(cfg(bilateral_radius=0), O.seed(0), D)
    l1 = out[1]["D"][..., 0]
    ys, xs = np.mgrid[0:H // 2, 0:W // 2]
    inner = (xs >= 1) & (ys >= 1) & (xs < W // 2 - 1) & (ys < H // 2 - 1)
    assert np.abs(l1 - D[2 * ys, 2 * xs])[inner].max() < 1e-14


@pytest.mark.parametrize("n", [np.array([0.0, 0.0, 1.0]), np.array([0.3, -0.2, 0.9]) / np.linalg.norm([0.3, -0.2, 0.9])])
def test_vertices_on_plane_and_normal_faces_camera(n):
    d = 1.5
    D, ray = plane_depth(n, d)
    lv = O.measure(cfg(bilateral_radius=0), O.seed(0), D)[0]
    V, N, valid = lv["V"][..., 0], lv["N"][..., 0], lv["valid"].astype(bool)
    assert np.abs(V @ n - d).max() < 1e-14
    assert valid[:-1, :-1].all() and not valid[-1].any() and not valid[:, -1].any()
    assert np.abs(N[valid] + n).max() < 1e-12   # -n points back at the camera


def test_vertex_derivatives_depth_and_focal_length():
    D = 1.0 + 0.3 * np.random.default_rng(1).random((H, W))
    _, ray = plane_depth(np.array([0, 0, 1.0]), 1.0)
    h = 1e-20
    lv = O.measure(cfg(bilateral_radius=0), O.seed(1, O.P_DEPTH, h=h), D, np.ones((H, W)))[0]
    assert np.allclose(lv["V"][..., 1] / h, ray, rtol=0, atol=1e-15)     # dV/dD = K^-1 (u,1)
    lv = O.measure(cfg(bilateral_radius=0), O.seed(1, O.P_FX, h=h), D)[0]
    xs = np.arange(W)[None, :]
    assert np.allclose(lv["V"][..., 0, 1] / h, -D * (xs - CX) / FX ** 2, rtol=1e-14, atol=1e-17)
    assert np.all(lv["V"][..., 1:, 1] == 0.0)
    # coarser level uses K / 2: same closed form with halved intrinsics
    l1 = O.measure(cfg(bilateral_radius=0), O.seed(1, O.P_FX, h=h), D)[1]
    D1 = l1["D"][..., 0]
    x1 = np.arange(W // 2)[None, :]
    ok = l1["valid"].astype(bool) | (D1 > 0)
    ref = -D1 * (x1 - CX / 2) / (FX / 2) ** 2 / 2   # d/dfx of (x - cx/2)/(fx/2)
    assert np.allclose((l1["V"][..., 0, 1] / h)[ok], ref[ok], rtol=1e-13, atol=1e-16)


def test_invalid_pixels_stay_invalid_and_zero():
    D = np.full((H, W), 1.2)
    D[5, 7] = 0.0
    D[10, 3] = np.nan
    lv = O.measure(cfg(), O.seed(0), D)[0]
    assert lv["D"][5, 7, 0] == 0.0 and lv["D"][10, 3, 0] == 0.0
    assert not lv["valid"][5, 7] and not lv["valid"][4, 7] and not lv["valid"][5, 6]
