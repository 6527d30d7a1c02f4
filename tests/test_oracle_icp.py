"""Pins of the oracle's projective point-to-plane ICP (Sec. 4.1 "Differentiable
ICP", eq. icp): zero motion is a fixed point; a known rigid motion of about
2 degrees and 3 cm is recovered from analytic model maps of a planar scene to
1e-9 when the model keeps only taps whose 2x2 lookup block lies on one face
(bilinear interpolation of coplanar points stays on the plane, so every
residual is the exact point-to-plane distance and Gauss-Newton converges to
the true pose), and to 0.2 mm with the face edges kept (blended taps at
creases); the complex solve of the normal equations equals the real solve
plus its first-order perturbation."""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle as O
import scenegen as sg

W, H = 160, 120
CAM = dict(fx=130.0, fy=130.0, cx=79.5, cy=59.5)


def cfg(**kw):
    d = dict(width=W, height=H, bilateral_radius=0, **CAM)
    d.update(kw)
    return O.config(None, **d)


def planar_scene():
    sc = sg.make_scene(0, 2.56)
    return sg.Scene(L=sc.L, floor_y=sc.floor_y, spheres=np.zeros((0, 4)),
                    boxes=np.array([[0.3, sc.floor_y + 0.3, 0.2, 0.3, 0.3, 0.25],
                                    [-0.4, sc.floor_y + 0.2, -0.3, 0.2, 0.2, 0.35]]))


def model_maps(scene, T):
    z, P, N = sg.render_maps(scene, T, W, H, **CAM)
    return dict(V=P[..., None], N=N[..., None], Z=z, valid=(z > 0).astype(np.uint8))


def coplanar_blocks(z, P, N):
    """Pixels whose 2x2 block (the pixel, its right, lower and diagonal
    neighbours) lies on one plane: equal normal n and offset n.p."""
    key = np.concatenate([N, np.einsum("hwi,hwi->hw", N, P)[..., None]], -1)
    ok = z > 0
    ok[-1, :] = False
    ok[:, -1] = False
    for dy, dx in ((0, 1), (1, 0), (1, 1)):
        nb = np.zeros_like(key)
        nb[:H - dy, :W - dx] = key[dy:, dx:]
        znb = np.zeros_like(z)
        znb[:H - dy, :W - dx] = z[dy:, dx:]
        ok &= (znb > 0) & (np.abs(nb - key).max(-1) <= 1e-9)
    return ok


def twist(xi):
    M = np.zeros((4, 4))
    M[0, 1], M[0, 2], M[1, 0], M[1, 2], M[2, 0], M[2, 1] = -xi[2], xi[1], xi[2], -xi[0], -xi[1], xi[0]
    M[:3, 3] = xi[3:]
    return M


def test_zero_motion_is_a_fixed_point():
    sc = planar_scene()
    T = sg.look_at((0.9, 0.2, -1.2), (0, sc.floor_y + 0.2, 0))
    s = O.seed(0)
    z, _, _ = sg.render_maps(sc, T, W, H, **CAM)
    lv = O.measure(cfg(), s, z)[0]
    model = dict(V=(lv["V"][..., 0] @ T[:3, :3].T + T[:3, 3])[..., None],
                 N=(lv["N"][..., 0] @ T[:3, :3].T)[..., None], Z=z, valid=lv["valid"])
    A, b, cnt, r2 = O.icp_reduce(cfg(), s, 0, lv, model, T[..., None], T[..., None])
    assert cnt > 0.3 * W * H
    assert np.abs(b[:, 0]).max() < 1e-12 * np.abs(A[:, 0]).max()
    Tout, lost, _, _ = O.track(cfg(iters=(10, 0, 0)), s, z, None, model, T[..., None], T[..., None])
    assert lost == 0
    assert np.abs(Tout[..., 0] - T).max() < 1e-12


@pytest.mark.parametrize("motion", [np.array([0.01, -0.02, 0.015, 0.02, -0.01, 0.03]),
                                    np.array([-0.03, 0.01, 0.0, -0.03, 0.02, 0.0])])
def test_known_motion_recovered_with_face_edges(motion):
    sc = planar_scene()
    Tprev = sg.look_at((0.9, 0.2, -1.2), (0, sc.floor_y + 0.2, 0))
    Tcur = expm(twist(motion)) @ Tprev
    s = O.seed(0)
    z, _, _ = sg.render_maps(sc, Tcur, W, H, **CAM)
    model = model_maps(sc, Tprev)
    Tout, lost, cnt, r2 = O.track(cfg(), s, z, None, model, Tprev[..., None], Tprev[..., None])
    assert lost == 0
    err_t = np.linalg.norm(Tout[:3, 3, 0] - Tcur[:3, 3])
    err_r = np.linalg.norm(Tout[:3, :3, 0] - Tcur[:3, :3])
    assert err_t < 2e-4 and err_r < 2e-4, (err_t, err_r)


@pytest.mark.parametrize("motion", [np.array([0.01, -0.02, 0.015, 0.02, -0.01, 0.03]),
                                    np.array([-0.03, 0.01, 0.0, -0.03, 0.02, 0.0])])
def test_known_motion_recovered_exactly_on_face_interiors(motion):
    sc = planar_scene()
    Tprev = sg.look_at((0.9, 0.2, -1.2), (0, sc.floor_y + 0.2, 0))
    Tcur = expm(twist(motion)) @ Tprev
    assert 1.5 <= np.degrees(np.linalg.norm(motion[:3])) <= 2.0
    assert 0.03 <= np.linalg.norm(motion[3:]) <= 0.04
    s = O.seed(0)
    z, _, _ = sg.render_maps(sc, Tcur, W, H, **CAM)
    zm, Pm, Nm = sg.render_maps(sc, Tprev, W, H, **CAM)
    model = dict(V=Pm[..., None], N=Nm[..., None], Z=zm, valid=coplanar_blocks(zm, Pm, Nm).astype(np.uint8))
    Tout, lost, cnt, r2 = O.track(cfg(), s, z, None, model, Tprev[..., None], Tprev[..., None])
    assert lost == 0 and cnt > 0.5 * W * H
    assert r2 < 1e-20
    err_t = np.linalg.norm(Tout[:3, 3, 0] - Tcur[:3, 3])
    err_r = np.linalg.norm(Tout[:3, :3, 0] - Tcur[:3, :3])
    assert err_t < 1e-9 and err_r < 1e-9, (err_t, err_r)


def test_complex_solve_is_real_solve_plus_first_order_perturbation():
    rng = np.random.default_rng(3)
    M = rng.standard_normal((6, 6))
    A0 = M @ M.T + 6 * np.eye(6)
    B = rng.standard_normal((6, 6))
    A1 = B + B.T
    b0, b1 = rng.standard_normal(6), rng.standard_normal(6)
    h = 1e-20
    s = O.seed(1, h=h)
    iu = np.triu_indices(6)
    A = np.stack([A0[iu], h * A1[iu]], -1)
    b = np.stack([b0, h * b1], -1)
    w = np.array([0.7, 0.0])
    x, lost = O.solve(s, A, b, w)
    assert lost == 0
    x0 = -np.linalg.solve(A0, b0)
    x1 = -np.linalg.solve(A0, b1 + A1 @ x0)
    assert np.allclose(x[:, 0], 0.7 * x0, rtol=1e-13, atol=1e-15)
    assert np.allclose(x[:, 1] / h, 0.7 * x1, rtol=1e-12, atol=1e-14)


def test_singular_normal_matrix_is_lost():
    s = O.seed(0)
    J = np.array([0, 0, 0, 0, 0, 1.0])
    A0 = np.outer(J, J)
    iu = np.triu_indices(6)
    _, lost = O.solve(s, A0[iu][:, None], np.zeros((6, 1)))
    assert lost == 1
