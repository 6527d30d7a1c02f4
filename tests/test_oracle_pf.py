"""Pins of the oracle's surfel front end (X-PointFusion, Sec. 4.2).

* the first frame inserts every valid measured pixel, in pixel order, with
  v = T V(u), n = R N(u), t = 0 and the confidence exp(-gamma^2 / 0.72) in
  closed form;
* the index map keeps the surfel nearest to the camera per sub-pixel (ties
  to the lower index), skips surfels under the confidence floor, and puts a
  surfel at a pixel centre in sub-pixel (2, 2) of that pixel's 4 x 4 block;
* a hand-built map around one pixel: the candidates within the three gates
  are all updated (one-to-many) with the Gaussian weight of their distance,
  v <- (c v + w C V) / (c + w C) etc. in closed form; a candidate beyond the
  depth gate or with a turned normal is left alone, and its pixel then gets
  a new surfel;
* the same frame again at the same pose: every surfel is updated once, by
  its own pixel, its position stays, its confidence doubles, nothing is
  inserted;
* the complex-step derivatives of the final pose and of surfel positions
  with respect to the initial pose agree with central differences of real
  runs.
"""
import numpy as np
import pytest

import oracle as O

W, H = 40, 30
FX = FY = 30.0
CX, CY = 19.5, 14.5


def cfg(**kw):
    d = dict(width=W, height=H, fx=FX, fy=FY, cx=CX, cy=CY, dim=(32,) * 3, voxel=0.02, trunc=0.06,
             bilateral_radius=0, iters=(6, 4, 0))
    d.update(kw)
    return O.config(None, **d)


def plane_depth(z0=1.0, tilt=0.0, tilt_y=0.0):
    u, v = np.meshgrid(np.arange(W, dtype=float), np.arange(H, dtype=float))
    rx, ry = (u - CX) / FX, (v - CY) / FY
    return z0 / (1.0 - tilt * rx - tilt_y * ry)   # the plane z = z0 + tilt x + tilt_y y (camera frame)


def stairs_depth(z0=1.2, tilt=0.3):
    """Three planes with independent normals: every pose direction is
    observable."""
    D = plane_depth(z0, tilt)
    D[:, 20:] = plane_depth(z0 - 0.1, 0.0, 0.4)[:, 20:]
    D[15:, :20] = plane_depth(z0 + 0.05, -tilt)[15:, :20]
    return D


def pose(tx=0.0, ty=0.0, tz=0.0):
    T = np.eye(4)
    T[:3, 3] = (tx, ty, tz)
    return T


def confidence(x, y):
    g2 = ((x - CX) ** 2 + (y - CY) ** 2) / (CX ** 2 + CY ** 2)
    return np.exp(-g2 / 0.72)


def test_first_frame_inserts_every_valid_pixel_in_order():
    c = cfg()
    s = O.seed(0)
    D = plane_depth(1.1, 0.3)
    T = pose(0.02, -0.01, -0.5)
    st = O.PfState(c, s, O.lift(T, s))
    stats, pf = O.pf_frame_step(c, s, st, D)
    m = O.measure(c, s, D)[0]
    valid = m["valid"].reshape(-1).astype(bool)
    idx = np.nonzero(valid)[0]
    S = st.surfels()
    assert pf[1] == valid.sum() == len(S["t"]) and pf[0] == 0 and pf[2] == 0
    V = m["V"][..., 0].reshape(-1, 3)[idx]
    N = m["N"][..., 0].reshape(-1, 3)[idx]
    assert np.abs(S["v"][:, :, 0] - (V @ T[:3, :3].T + T[:3, 3])).max() < 1e-14
    assert np.abs(S["n"][:, :, 0] - N @ T[:3, :3].T).max() < 1e-14
    x, y = idx % W, idx // W
    assert np.abs(S["c"][:, 0] - confidence(x, y)).max() < 1e-14
    nz = np.maximum(np.abs(N[:, 2]), 0.25)
    assert np.abs(S["r"][:, 0] - np.sqrt(2.0) * V[:, 2] / (FX * nz)).max() < 1e-14
    assert np.all(S["t"] == 0)


def test_index_map_nearest_ties_confidence_floor_and_centre_subpixel():
    c = cfg()
    T = pose()
    # pixel (10, 7) centre direction at depth 1 and 2; a third surfel at the
    # same depth as the first (a tie), a fourth under the confidence floor
    ray = np.array([(10 - CX) / FX, (7 - CY) / FY, 1.0])
    v = np.stack([1.0 * ray, 0.5 * ray, 0.5 * ray, 0.25 * ray, 2.0 * ray])
    conf = np.array([1.0, 1.0, 1.0, 0.1, 1.0])
    idx = O.pf_index_map(c, v, conf, T, sup=4, c_min=0.5)
    q = (7 * 4 + 2, 10 * 4 + 2)
    assert idx[q] == 1                       # nearest; the tie (index 2) keeps the lower index
    assert (idx >= 0).sum() == 1
    idx1 = O.pf_index_map(c, v, conf, T, sup=1, c_min=0.0)
    assert idx1[7, 10] == 3 and (idx1 >= 0).sum() == 1


def test_one_to_many_update_and_gates():
    c = cfg(pf_d_depth=0.03, pf_d_norm_deg=30.0, pf_d_dist=0.03, pf_sigma=0.015)
    s = O.seed(0)
    D = plane_depth(1.0)
    T = pose()
    m = O.measure(c, s, D)[0]
    u0, u1 = (7, 10), (12, 20)      # (y, x)
    V0 = m["V"][u0][:, 0]
    N0 = m["N"][u0][:, 0]
    V1 = m["V"][u1][:, 0]
    N1 = m["N"][u1][:, 0]
    # A, B: within every gate, different sub-pixels of u0's block; C: beyond
    # the depth gate (alone in u1's block); E: u0's block, normal turned 90 deg
    pts = np.stack([V0 + [0.006, 0.0, 0.0], V0 + [-0.006, 0.0, 0.001], V1 + [0.0, 0.0, 0.04],
                    V0 + [0.0, -0.006, 0.0]])
    nrm = np.stack([N0, N0, N1, np.cross(N0, [1.0, 0.0, 0.0])])
    nrm[3] /= np.linalg.norm(nrm[3])
    conf = np.array([1.5, 0.7, 2.0, 1.0])
    rad = np.array([0.01, 0.02, 0.03, 0.04])
    idx = O.pf_index_map(c, pts, conf, T, sup=4)
    where = {int(i): np.argwhere(idx == i)[0] // 4 for i in range(4)}
    assert tuple(where[0]) == u0 and tuple(where[1]) == u0 and tuple(where[3]) == u0 and tuple(where[2]) == u1
    assert len({tuple(np.argwhere(idx == i)[0]) for i in range(4)}) == 4
    st = O.PfState(c, s, O.lift(T, s))
    st.S["v"][:4, :, 0] = pts
    st.S["n"][:4, :, 0] = nrm
    st.S["c"][:4, 0] = conf
    st.S["r"][:4, 0] = rad
    st.S["t"][:4] = -5
    st.count[0] = 4
    stats, pf = O.pf_frame_step(c, s, st, D)
    valid = m["valid"].astype(bool)
    assert pf[0] == 2 and pf[1] == valid.sum() - 1
    S = st.surfels()
    Cu = confidence(u0[1], u0[0])
    r_new = np.sqrt(2.0) * V0[2] / (FX * max(abs(N0[2]), 0.25))
    for i in (0, 1):
        d2 = np.sum((pts[i] - V0) ** 2)
        a = np.exp(-d2 / (2 * 0.015 ** 2)) * Cu
        den = conf[i] + a
        assert np.abs(S["v"][i, :, 0] - (conf[i] * pts[i] + a * V0) / den).max() < 1e-14
        assert np.abs(S["n"][i, :, 0] - (conf[i] * nrm[i] + a * N0) / den).max() < 1e-14
        assert abs(S["c"][i, 0] - den) < 1e-14
        assert abs(S["r"][i, 0] - (conf[i] * rad[i] + a * r_new) / den) < 1e-14
        assert S["t"][i] == 0
    for i in (2, 3):
        assert np.array_equal(S["v"][i, :, 0], pts[i]) and S["c"][i, 0] == conf[i] and S["t"][i] == -5
    # u1's only candidate failed a gate: u1 got a new surfel (in pixel order)
    new = S["v"][4:, :, 0]
    order = [q for q in np.flatnonzero(valid.reshape(-1)) if q != u0[0] * W + u0[1]]
    k1 = order.index(u1[0] * W + u1[1])
    assert np.abs(new[k1] - V1).max() < 1e-15


def test_same_frame_again_doubles_confidence_and_keeps_positions():
    c = cfg(iters=(0, 0, 0))          # no ICP pass: the second frame is at the same pose
    s = O.seed(0)
    D = stairs_depth(1.2, 0.2)
    T = pose(0.01, 0.0, -0.3)
    st = O.PfState(c, s, O.lift(T, s))
    O.pf_frame_step(c, s, st, D)
    S0 = {k: v.copy() for k, v in st.surfels().items()}
    stats, pf = O.pf_frame_step(c, s, st, D)
    S1 = st.surfels()
    assert stats[0] == 0 and np.array_equal(st.T1[:, :, 0], T)
    assert pf[1] == 0 and pf[0] == len(S0["t"])
    assert np.abs(S1["v"] - S0["v"]).max() < 1e-12
    assert np.abs(S1["c"][:, 0] - 2.0 * S0["c"][:, 0]).max() < 1e-12
    assert np.all(S1["t"] == 1)


def test_pose_derivatives_match_central_differences():
    from scipy.linalg import expm
    c = cfg()
    D = np.stack([stairs_depth(1.2, 0.3), stairs_depth(1.19, 0.3), stairs_depth(1.18, 0.31)])
    T0 = pose(0.01, 0.02, -0.4)
    h = 1e-20
    for a in (0, 4):                                # phi_x, rho_y
        rc = O.pf_run_sequence(c, O.seed(1, a, h=h), D, T0)
        eps = 1e-6
        xi = np.zeros(6)
        xi[a] = eps
        Xh = np.zeros((4, 4))
        Xh[:3, :3] = [[0, -xi[2], xi[1]], [xi[2], 0, -xi[0]], [-xi[1], xi[0], 0]]
        Xh[:3, 3] = xi[3:]
        rp = O.pf_run_sequence(c, O.seed(0), D, expm(Xh) @ T0)
        rm = O.pf_run_sequence(c, O.seed(0), D, expm(-Xh) @ T0)
        assert len(rp["surfels"]["t"]) == len(rm["surfels"]["t"]) == len(rc["surfels"]["t"])
        assert np.array_equal(rp["pf"], rc["pf"]) and np.array_equal(rm["pf"], rc["pf"])
        dT = rc["poses"][-1][..., 1] / h
        dT_fd = (rp["poses"][-1][..., 0] - rm["poses"][-1][..., 0]) / (2 * eps)
        assert np.abs(dT - dT_fd).max() <= 1e-5 * max(np.abs(dT).max(), 1.0)
        dv = rc["surfels"]["v"][..., 1] / h
        dv_fd = (rp["surfels"]["v"][..., 0] - rm["surfels"]["v"][..., 0]) / (2 * eps)
        assert np.abs(dv - dv_fd).max() <= 1e-5 * np.abs(dv).max()
