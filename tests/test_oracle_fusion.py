"""Pins of the oracle's TSDF fusion (Sec. 4.1 "Surface Update") on a
fronto-parallel plane, where the projective signed distance, its truncation
and its derivatives have closed forms, and on repeated identical frames (the
running average is a fixed point; the weight saturates at the cap)."""
import numpy as np
import pytest

import oracle as O

W, H = 40, 30
DIM, VOX = 32, 0.02   # 0.64 m cube
MU = 0.06
DEPTH = 1.2           # plane at world z = 0.2 seen from z = -1


def cfg(**kw):
    d = dict(width=W, height=H, fx=30.0, fy=30.0, cx=19.5, cy=14.5, dim=(DIM,) * 3, voxel=VOX,
             trunc=MU, wcap=64.0, bilateral_radius=0)
    d.update(kw)
    return O.config(None, **d)


def pose():
    T = np.eye(4)
    T[2, 3] = -1.0
    return T


def centres():
    i = np.arange(DIM ** 3)
    x, y, z = i % DIM, (i // DIM) % DIM, i // DIM ** 2
    c = (np.stack([x, y, z], -1) + 0.5) * VOX - 0.5 * DIM * VOX
    return c


def fuse_once(s, c=None, F=None, Wt=None, T=None):
    c = cfg() if c is None else c
    nc = O.ncomp(s)
    n = DIM ** 3
    F = np.zeros((n, nc)) if F is None else F
    Wt = np.zeros((n, nc)) if Wt is None else Wt
    Df = O.lift(np.full((H, W), DEPTH), s)
    T = O.lift(pose(), s) if T is None else T
    return O.fuse(c, s, F, Wt, Df, T)


def test_plane_tsdf_closed_form_and_update_set():
    F, Wt, n = fuse_once(O.seed(0))
    xz = centres()[:, 2] + 1.0
    eta = DEPTH - xz
    upd = Wt[:, 0] > 0
    assert n == upd.sum() > 0
    ref = np.clip(eta / MU, -1.0, 1.0)
    assert np.abs(F[upd, 0] - ref[upd]).max() < 1e-14
    assert np.all(eta[upd] >= -MU - 1e-12)           # behind the band: never updated
    assert not np.any(upd & (eta < -MU - 1e-12))


def test_plane_tsdf_derivatives():
    h = 1e-20
    xz = centres()[:, 2] + 1.0
    eta = DEPTH - xz
    band = np.abs(eta) < MU - 1e-9
    sat = eta > MU + 1e-9
    # truncation distance: dF/dmu = -eta/mu^2 in band, 0 when saturated
    F, Wt, _ = fuse_once(O.seed(1, O.P_TRUNC, h=h))
    upd = Wt[:, 0] > 0
    g = F[:, 1] / h
    assert np.allclose(g[upd & band], (-eta / MU ** 2)[upd & band], rtol=1e-12)
    assert np.all(g[upd & sat] == 0.0)
    # camera moved along +z (left-multiplied seed): dF/drho_z = 1/mu in band
    s = O.seed(1, O.P_RHO_Z, h=h)
    T = O.lift(pose(), s)
    T[2, 3, 1] = h
    F, Wt, _ = fuse_once(s, T=T)
    g = F[:, 1] / h
    assert np.allclose(g[upd & band], 1.0 / MU, rtol=1e-12)
    assert np.all(g[upd & sat] == 0.0)
    # focal length: constant depth => exactly zero
    F, Wt, _ = fuse_once(O.seed(1, O.P_FX, h=h))
    assert np.all(F[:, 1] == 0.0)


def test_identical_frames_fixed_point_and_weight_cap():
    cap = 5.0
    h = 1e-20
    s = O.seed(1, O.P_WCAP, h=h)
    c = cfg(wcap=cap)
    F = Wt = None
    first = None
    for k in range(8):
        F, Wt, _ = fuse_once(s, c, F, Wt)
        if first is None:
            first = F.copy()
            upd = Wt[:, 0] > 0
        # running average of equal values (up to the rounding of (W F + F)/(W + 1))
        assert np.abs(F[:, 0] - first[:, 0]).max() <= 4e-16
        g = F[:, 1] / h
        if k + 1 < cap:
            assert np.all(g == 0.0)                          # dF/dWcap = 0 exactly before the cap
        else:
            assert np.abs(g).max() <= 1e-15                  # (F - F_D) dW/(W+1): rounding only
        assert np.all(Wt[upd, 0] == min(k + 1, cap))
        dW = Wt[upd, 1] / h
        assert np.all(dW == (1.0 if k + 1 >= cap else 0.0))  # dW/dWcap is 0 until the cap binds


def test_fuse_margin_is_the_update_test():
    """The margin diagnostic (re eta + re mu for voxels reaching the update
    test) equals the plane's closed form and is >= 0 exactly on the updated
    voxels."""
    s = O.seed(0)
    F, Wt, n = fuse_once(s)
    idx = np.arange(DIM ** 3)
    m = O.fuse_margin(cfg(), s, O.lift(np.full((H, W), DEPTH), s), O.lift(pose(), s), idx)
    upd = Wt[:, 0] > 0
    reach = ~np.isnan(m)
    assert np.array_equal(upd, reach & (m >= 0))
    eta = DEPTH - (centres()[:, 2] + 1.0)
    assert np.abs(m[reach] - (eta[reach] + MU)).max() < 1e-14
