"""Pins of the oracle's raycast (Sec. 4.1 "Ray casting", eq. surface_prediction)
on an analytic planar TSDF.  With F linear in space, trilinear interpolation and
the linear zero-crossing formula are exact, so the predicted vertex, normal and
their CSFD derivatives with respect to the pose and the focal length must equal
the ray-plane intersection in closed form."""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle as O

W, H = 40, 30
FX, FY, CX, CY = 30.0, 31.0, 19.5, 14.5
DIM, VOX, MU = 48, 0.02, 0.06
NRM = np.array([0.1, 0.2, 1.0]) / np.linalg.norm([0.1, 0.2, 1.0])
DPL = 0.05


def cfg():
    return O.config(None, width=W, height=H, fx=FX, fy=FY, cx=CX, cy=CY, dim=(DIM,) * 3, voxel=VOX,
                    trunc=MU, bilateral_radius=0)


def planar_volume(s):
    i = np.arange(DIM ** 3)
    c = (np.stack([i % DIM, (i // DIM) % DIM, i // DIM ** 2], -1) + 0.5) * VOX - 0.5 * DIM * VOX
    F = (DPL - c @ NRM) / MU
    return O.lift(F, s), O.lift(np.ones(DIM ** 3), s)


def pose():
    T = np.eye(4)
    T[:3, :3] = expm(np.array([[0, -0.05, 0.03], [0.05, 0, -0.04], [-0.03, 0.04, 0]]))
    T[:3, 3] = [0.03, -0.02, -0.9]
    return T


def closed_form(T, fx=FX):
    x = (np.arange(W) - CX) / fx
    y = (np.arange(H) - CY) / FY
    dh = np.stack(np.broadcast_arrays(x[None, :], y[:, None], np.ones((1, 1))), -1)
    dirs = dh @ T[:3, :3].T
    t = T[:3, 3]
    a0 = (DPL - NRM @ t) / (dirs @ NRM)
    return a0, t + a0[..., None] * dirs, dirs


def test_planar_hit_and_normal_exact():
    s = O.seed(0)
    F, Wt = planar_volume(s)
    out = O.raycast(cfg(), s, F, Wt, O.lift(pose(), s))
    a0, V, _ = closed_form(pose())
    ok = out["valid"].astype(bool)
    assert ok.sum() > 0.5 * W * H
    assert np.abs(out["V"][..., 0][ok] - V[ok]).max() < 1e-13
    assert np.abs(out["Z"][ok] - a0[ok]).max() < 1e-13
    assert np.abs(out["N"][..., 0][ok] + NRM).max() < 1e-13


@pytest.mark.parametrize("d", [3, 4, 5])
def test_planar_hit_translation_derivative(d):
    h = 1e-20
    s = O.seed(1, d, h=h)
    F, Wt = planar_volume(s)
    T = O.lift(pose(), s)
    T[d - 3, 3, 1] = h   # left-multiplied translation seed = world translation
    out = O.raycast(cfg(), s, F, Wt, T)
    a0, V, dirs = closed_form(pose())
    da = -NRM[d - 3] / (dirs @ NRM)
    dV = da[..., None] * dirs
    dV[..., d - 3] += 1.0
    ok = out["valid"].astype(bool)
    assert np.abs(out["V"][..., 1][ok] / h - dV[ok]).max() < 1e-12
    assert np.abs(out["N"][..., 1][ok] / h).max() < 1e-12   # plane normal does not move


def test_planar_hit_focal_length_derivative():
    h = 1e-20
    s = O.seed(1, O.P_FX, h=h)
    F, Wt = planar_volume(s)
    out = O.raycast(cfg(), s, F, Wt, O.lift(pose(), s))
    a0, V, dirs = closed_form(pose())
    x = (np.arange(W) - CX)
    ddh = np.zeros((H, W, 3))
    ddh[..., 0] = -x[None, :] / FX ** 2
    ddirs = ddh @ pose()[:3, :3].T
    da = -a0 * (ddirs @ NRM) / (dirs @ NRM)
    dV = da[..., None] * dirs + a0[..., None] * ddirs
    ok = out["valid"].astype(bool)
    assert np.abs(out["V"][..., 1][ok] / h - dV[ok]).max() < 1e-12


def test_unobserved_volume_gives_no_hits_and_pixel_list_matches_full():
    s = O.seed(0)
    F, Wt = planar_volume(s)
    out = O.raycast(cfg(), s, F, np.zeros_like(Wt), O.lift(pose(), s))
    assert not out["valid"].any()
    full = O.raycast(cfg(), s, F, Wt, O.lift(pose(), s))
    pix = np.array([0, 17, 333, W * H - 1, 611], dtype=np.int32)
    part = O.raycast(cfg(), s, F, Wt, O.lift(pose(), s), pix=pix)
    assert np.array_equal(part["V"], full["V"].reshape(-1, 3, 1)[pix])
    assert np.array_equal(part["valid"], full["valid"].reshape(-1)[pix])
