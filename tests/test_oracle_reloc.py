"""Pins of the oracle's camera relocalisation objective (Sec. 5.2):
E(T_q) = sum over voxels of (F_r - F_q)^2, F_q the reference volume after the
query depth is fused into it at T_q.

* the definition: E equals the sum of squared changes that the oracle's own
  fusion (pinned in test_oracle_fusion.py) makes to the observed voxels, and
  the count equals the number of observed voxels it updates;
* a reference fused from the query's own depth at the query's pose: E, and
  its gradient, are exactly zero there, and E grows away from it;
* a fronto-parallel plane with an arbitrary reference volume and a pure
  translation, where E, g and the rho_z row of H have closed forms from the
  chain rule (d eta / d rho_z = 1, d eta / d phi = (c_y, -c_x, 0), none on
  rho_x, rho_y, phi_z);
* the gradient and Hessian against central differences of E and of g on a
  tilted plane.
"""
import numpy as np
import pytest

import oracle as O

W, H = 40, 30
DIM, VOX = 32, 0.02   # 0.64 m cube centred at the origin
MU = 0.06
FX = FY = 30.0
CX, CY = 19.5, 14.5


def cfg(**kw):
    d = dict(width=W, height=H, fx=FX, fy=FY, cx=CX, cy=CY, dim=(DIM,) * 3, voxel=VOX, trunc=MU, wcap=64.0,
             bilateral_radius=0)
    d.update(kw)
    return O.config(None, **d)


def centres():
    i = np.arange(DIM ** 3)
    x, y, z = i % DIM, (i // DIM) % DIM, i // DIM ** 2
    return (np.stack([x, y, z], -1) + 0.5) * VOX - 0.5 * DIM * VOX


def trans(x, y, z):
    T = np.eye(4)
    T[:3, 3] = (x, y, z)
    return T


def rot(axis, ang):
    a = np.asarray(axis, float)
    a /= np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    R = np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K
    T = np.eye(4)
    T[:3, :3] = R
    return T


def tilted_plane_depth(T):
    """Depth image of the world plane z = 0.1 + 0.2 x + 0.1 y seen from the
    camera-to-world pose T (ray-plane intersection per pixel centre)."""
    u, v = np.meshgrid(np.arange(W, dtype=float), np.arange(H, dtype=float))
    r = np.stack([(u - CX) / FX, (v - CY) / FY, np.ones_like(u)], -1)
    d = r @ T[:3, :3].T
    o = T[:3, 3]
    n = np.array([-0.2, -0.1, 1.0])
    lam = (0.1 - n @ o) / (d @ n)
    return lam   # the camera z of the hit is lam (r has unit z)


def reference(c, depths_poses):
    s = O.seed(0)
    n = DIM ** 3
    F, Wt = np.zeros((n, 1)), np.zeros((n, 1))
    for D, T in depths_poses:
        F, Wt, _ = O.fuse(c, s, F, Wt, D[..., None], T[..., None])
    return F[:, 0], Wt[:, 0]


def test_energy_is_the_sum_of_squared_changes_fusion_makes():
    c = cfg()
    T1, T2 = trans(0, 0, -1.0), rot([0, 1, 0], 0.05) @ trans(0.03, -0.02, -1.02)
    F, Wt = reference(c, [(tilted_plane_depth(T1), T1), (tilted_plane_depth(T2), T2)])
    assert (Wt == 2).sum() > 1000
    Tq = rot([1, 0.3, 0.2], 0.03) @ trans(0.012, 0.007, -0.985)
    Dq = tilted_plane_depth(trans(0.01, 0.0, -0.99))     # not the depth of Tq: E > 0
    E, g, Hs, cnt = O.reloc_energy(c, F, Wt, Dq, Tq, order=0)
    Ff, Wf, _ = O.fuse(c, O.seed(0), F[:, None], Wt[:, None], Dq[..., None], Tq[..., None])
    obs = Wt > 0
    upd = obs & (Wf[:, 0] != Wt)
    E_def = np.sum((F[obs] - Ff[obs, 0]) ** 2)
    assert cnt == upd.sum() > 500
    assert E > 0
    assert abs(E - E_def) <= 1e-12 * E_def
    assert np.all(g == 0) and np.all(Hs == 0)      # order 0


def test_zero_at_the_pose_the_reference_was_fused_from():
    c = cfg()
    T = rot([0.2, 1, 0], 0.04) @ trans(0.01, 0.02, -1.0)
    D = tilted_plane_depth(T)
    F, Wt = reference(c, [(D, T)])
    E, g, Hs, cnt = O.reloc_energy(c, F, Wt, D, T, order=2)
    assert cnt > 1000
    assert E == 0.0
    assert np.all(g == 0.0)
    ev = np.linalg.eigvalsh(Hs)
    assert ev.max() > 0 and ev.min() >= -1e-12 * ev.max()   # a minimum: H = 2 sum grad d grad d^T
    for k in range(6):
        xi = np.zeros(6)
        xi[k] = 2e-3
        from scipy.linalg import expm
        Xh = np.zeros((4, 4))
        Xh[:3, :3] = [[0, -xi[2], xi[1]], [xi[2], 0, -xi[0]], [-xi[1], xi[0], 0]]
        Xh[:3, 3] = xi[3:]
        assert O.reloc_energy(c, F, Wt, D, expm(Xh) @ T, order=0)[0] > 0


@pytest.mark.parametrize("w", [1.0, 3.0])
def test_fronto_parallel_plane_closed_form(w):
    c = cfg()
    d0 = 1.05
    Df = np.full((H, W), d0)
    cc = centres()
    rng = np.random.default_rng(5)
    Fr = np.tanh((0.08 - cc[:, 2]) / MU) + 0.05 * rng.standard_normal(len(cc))
    Wr = np.where(rng.random(len(cc)) < 0.8, w, 0.0)
    tx, ty, tz = 0.0013, -0.0021, -0.9937
    Tq = trans(tx, ty, tz)
    E, g, Hs, cnt = O.reloc_energy(c, Fr, Wr, Df, Tq, order=2)
    # closed form: x = c - t, u = fx x/z + cx, L = d0, eta = d0 - x_z
    x = cc - np.array([tx, ty, tz])
    z = x[:, 2]
    u = FX * x[:, 0] / z + CX
    v = FY * x[:, 1] / z + CY
    fu, fv = np.floor(u), np.floor(v)
    inview = (z > 0) & (fu >= 0) & (fv >= 0) & (fu <= W - 2) & (fv <= H - 2)
    eta = d0 - z
    sel = (Wr > 0) & inview & (eta >= -MU)
    band = sel & (eta < MU)
    Fd = np.where(eta >= MU, 1.0, eta / MU)
    dv = (Fr - Fd) / (Wr + 1.0)
    E_cf = np.sum(dv[sel] ** 2)
    # d d / d(phi_x, phi_y, phi_z, rho_x, rho_y, rho_z) in the band
    k = -1.0 / ((Wr + 1.0) * MU)
    J = np.zeros((len(cc), 6))
    J[:, 0] = k * cc[:, 1]
    J[:, 1] = -k * cc[:, 0]
    J[:, 5] = k
    g_cf = 2 * (J[band] * dv[band, None]).sum(0)
    assert cnt == sel.sum() > 1000
    assert abs(E - E_cf) <= 1e-12 * E_cf
    assert np.abs(g - g_cf).max() <= 1e-9 * np.abs(g_cf).max()
    assert np.abs(g[2:5]).max() <= 1e-13 * np.abs(g).max()   # phi_z, rho_x, rho_y leave eta alone
    # rho_z enters eta linearly: H_zz = 2 sum (d d/d rho_z)^2, and the mixed
    # phi_x / phi_y - rho_z terms have no second derivative of eta
    assert abs(Hs[5, 5] - 2 * np.sum(J[band, 5] ** 2)) <= 1e-10 * Hs[5, 5]
    for a in (0, 1):
        ref = 2 * np.sum(J[band, a] * J[band, 5])
        assert abs(Hs[a, 5] - ref) <= 1e-9 * abs(ref)
    # eta has no second derivative in (rho_x, rho_y) with each other, with
    # rho_z or with phi_z (the increment's rho / phi coupling, [phi]x rho / 2,
    # reaches x_z only through phi_x, phi_y)
    for a, b in ((3, 3), (4, 4), (3, 4), (3, 5), (4, 5), (2, 3), (2, 4), (2, 5)):
        assert abs(Hs[a, b]) <= 1e-13 * np.abs(Hs).max()


def test_gradient_and_hessian_against_central_differences():
    from scipy.linalg import expm
    c = cfg()
    T1, T2 = trans(0, 0, -1.0), rot([0, 1, 0], 0.05) @ trans(0.03, -0.02, -1.02)
    F, Wt = reference(c, [(tilted_plane_depth(T1), T1), (tilted_plane_depth(T2), T2)])
    Tq = rot([1, 0.3, 0.2], 0.02) @ trans(0.008, 0.005, -0.99)
    Dq = tilted_plane_depth(T1)
    E, g, Hs, cnt = O.reloc_energy(c, F, Wt, Dq, Tq, order=2)

    def at(xi):
        Xh = np.zeros((4, 4))
        Xh[:3, :3] = [[0, -xi[2], xi[1]], [xi[2], 0, -xi[0]], [-xi[1], xi[0], 0]]
        Xh[:3, 3] = xi[3:]
        return expm(Xh) @ Tq

    h = 1e-6
    gfd = np.zeros(6)
    Hfd = np.zeros((6, 6))
    for a in range(6):
        e = np.zeros(6)
        e[a] = h
        Ep, gp, _, cp = O.reloc_energy(c, F, Wt, Dq, at(e), order=1)
        Em, gm, _, cm = O.reloc_energy(c, F, Wt, Dq, at(-e), order=1)
        assert cp == cnt == cm          # no gate flips inside the stencil
        gfd[a] = (Ep - Em) / (2 * h)
        Hfd[:, a] = (gp - gm) / (2 * h)
    assert np.abs(g - gfd).max() <= 1e-6 * np.abs(g).max()
    # the derivative of g at exp(e) T is taken in a moving frame: the
    # left-increment Hessian equals its symmetric part
    Hsym = 0.5 * (Hfd + Hfd.T)
    assert np.abs(Hs - Hsym).max() <= 1e-4 * np.abs(Hs).max()
