"""End-to-end pins of the oracle's frame loop (Sec. 4.1 stage order):

* the CSFD derivative of every pose equals central finite differences of the
  real algorithm over a sweep of steps (runs whose decisions differ from the
  base run are discarded; the raycast's real-valued march schedule is held at
  the base run's, which is what the complex run does);
* hard gates and the weight cap before it binds give exactly zero derivatives;
* the bicomplex mixed second derivative is symmetric and matches finite
  differences of first derivatives (eq. csfd_hessian);
* the trajectory error and its derivative have closed forms for known offsets.
"""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle as O
import scenegen as sg

N_FRAMES = 4


def small_cfg(**kw):
    # 80x60 tracks reliably on two pyramid levels (a 20x15 third level does not)
    d = dict(width=80, height=60, fx=65.0, fy=65.0, cx=39.5, cy=29.5, dim=(96, 96, 96), voxel=0.0267,
             trunc=0.08, wcap=64.0, iters=(6, 4, 0))
    d.update(kw)
    return O.config(None, **d)


_SEQ = {}


def small_seq():
    if not _SEQ:
        p = sg.preset("c0")
        scene = sg.make_scene(p["seed"], p["L"])
        poses = sg.circle_trajectory(N_FRAMES, 1.5, 0.0, 2.0)
        seq = sg.Sequence(scene=scene, poses_gt=poses,
                          camera=dict(width=80, height=60, fx=65.0, fy=65.0, cx=39.5, cy=29.5),
                          seed=p["seed"], depth_dtype=np.float64)
        _SEQ["d"] = seq.depths()
        _SEQ["T0"] = poses[0]
        _SEQ["gt"] = poses
    return _SEQ["d"], _SEQ["T0"], _SEQ["gt"]


def twist(xi):
    M = np.zeros((4, 4))
    M[0, 1], M[0, 2], M[1, 0], M[1, 2], M[2, 0], M[2, 1] = -xi[2], xi[1], xi[2], -xi[0], -xi[1], xi[0]
    M[:3, 3] = xi[3:]
    return M


FIELD = {O.P_TRUNC: "trunc", O.P_FX: "fx", O.P_DGATE: "dgate", O.P_WCAP: "wcap", O.P_CY: "cy"}


def run_real(param, value_shift, base_poses, base_c):
    depths, T0, _ = small_seq()
    kw = {}
    T0p = T0
    if param < 6:
        e = np.zeros(6)
        e[param] = value_shift
        T0p = expm(twist(e)) @ T0
    else:
        kw[FIELD[param]] = getattr(base_c, FIELD[param]) + value_shift
    c = small_cfg(**kw)
    sched = np.array([base_c.trunc, base_c.fx, base_c.fy, base_c.cx, base_c.cy])
    return O.run_sequence(c, O.seed(0), depths, T0p, sched_poses=base_poses, sched_params=sched)


@pytest.mark.parametrize("param", [O.P_TRUNC, O.P_FX, O.P_CY, O.P_RHO_X, O.P_PHI_Y])
def test_csfd_matches_central_differences(param):
    depths, T0, _ = small_seq()
    c = small_cfg()
    base = O.run_sequence(c, O.seed(0), depths, T0)
    h = 1e-20
    cs = O.run_sequence(c, O.seed(1, param, h=h), depths, T0)
    g = cs["poses"][..., 1] / h
    assert np.array_equal(cs["poses"][..., 0], base["poses"][..., 0]) or \
        np.abs(cs["poses"][..., 0] - base["poses"][..., 0]).max() < 1e-15
    scale = np.abs(g).max()
    assert scale > 0
    best = np.inf
    for dlt in [1e-4, 3e-5, 1e-5, 3e-6, 1e-6, 3e-7, 1e-7, 3e-8]:
        rp = run_real(param, +dlt, base["poses"][..., 0], c)
        rm = run_real(param, -dlt, base["poses"][..., 0], c)
        same = (np.array_equal(rp["stats"][:, [0, 1, 3, 4, 5]], base["stats"][:, [0, 1, 3, 4, 5]]) and
                np.array_equal(rm["stats"][:, [0, 1, 3, 4, 5]], base["stats"][:, [0, 1, 3, 4, 5]]))
        if not same:
            continue
        fd = (rp["poses"][..., 0] - rm["poses"][..., 0]) / (2 * dlt)
        best = min(best, np.abs(fd - g).max() / scale)
    assert best <= 1e-6, best


@pytest.mark.parametrize("param", [O.P_DGATE, O.P_AGATE, O.P_WCAP])
def test_gates_and_unreached_cap_have_exactly_zero_derivative(param):
    depths, T0, _ = small_seq()
    cs = O.run_sequence(small_cfg(), O.seed(1, param, h=1e-20), depths, T0, want_volume=True)
    assert np.all(cs["poses"][..., 1] == 0.0)
    assert np.all(cs["F"][:, 1] == 0.0) and np.all(cs["W"][:, 1] == 0.0)


def test_hessian_symmetric_and_matches_fd_of_gradient():
    depths, T0, _ = small_seq()
    c = small_cfg()
    h = 1e-20
    a = O.run_sequence(c, O.seed(2, O.P_TRUNC, O.P_FX, h), depths, T0)["poses"]
    b = O.run_sequence(c, O.seed(2, O.P_FX, O.P_TRUNC, h), depths, T0)["poses"]
    Ha, Hb = a[..., 3] / h ** 2, b[..., 3] / h ** 2
    scale = np.abs(Ha).max()
    assert scale > 0
    assert np.abs(Ha - Hb).max() <= 1e-10 * scale
    # first-order parts of the bicomplex run equal the complex runs
    g1 = O.run_sequence(c, O.seed(1, O.P_TRUNC, h=h), depths, T0)["poses"][..., 1]
    assert np.abs(a[..., 1] - g1).max() <= 1e-12 * np.abs(g1).max()
    # d/dfx of dT/dmu by central differences of complex runs, with the real
    # march schedule held at the base run's (as inside the bicomplex run)
    base = O.run_sequence(c, O.seed(0), depths, T0)["poses"][..., 0]
    sched = np.array([c.trunc, c.fx, c.fy, c.cx, c.cy])
    best = np.inf
    for dlt in [1e-5, 3e-6, 1e-6, 3e-7]:
        gp = O.run_sequence(small_cfg(fx=c.fx + dlt), O.seed(1, O.P_TRUNC, h=h), depths, T0,
                            sched_poses=base, sched_params=sched)
        gm = O.run_sequence(small_cfg(fx=c.fx - dlt), O.seed(1, O.P_TRUNC, h=h), depths, T0,
                            sched_poses=base, sched_params=sched)
        fd = (gp["poses"][..., 1] - gm["poses"][..., 1]) / h / (2 * dlt)
        best = min(best, np.abs(fd - Ha).max() / scale)
    assert best <= 1e-5, best


def test_trajectory_error_closed_form():
    rng = np.random.default_rng(5)
    gt = np.tile(np.eye(4), (7, 1, 1))
    gt[:, :3, 3] = rng.standard_normal((7, 3))
    off = rng.standard_normal((7, 3)) * 0.01
    h = 1e-20
    s = O.seed(1, h=h)
    P = O.lift(gt, s)
    P[:, :3, 3, 0] += off
    P[:, :3, 3, 1] = h * off          # tangent along the offsets
    E = O.traj_err(s, P, gt)
    ref = np.sqrt(np.mean(np.sum(off ** 2, -1)))
    assert E[0] == pytest.approx(ref, rel=1e-14)
    assert E[1] / h == pytest.approx(ref, rel=1e-13)   # E is 1-homogeneous in the offsets


@pytest.mark.parametrize("pair", [(O.P_TRUNC, O.P_TRUNC), (O.P_TRUNC, O.P_FX), (O.P_RHO_X, O.P_CY)])
def test_bicomplex_and_complex_runs_share_the_real_run(pair):
    """Sec. 3: the real part of a complex-step evaluation is f(x) up to O(h^2),
    i.e. exactly f(x) in FP64 at h = 1e-20.  Every decision (validity, taps,
    gates, update masks) is taken on real parts, so complex and bicomplex runs
    must reproduce the real run bit for bit: poses, TSDF, weights and counts."""
    depths, T0, _ = small_seq()
    c = small_cfg()
    r0 = O.run_sequence(c, O.seed(0), depths, T0, want_volume=True)
    rc = O.run_sequence(c, O.seed(1, pair[0], h=1e-20), depths, T0, want_volume=True)
    rb = O.run_sequence(c, O.seed(2, pair[0], pair[1], 1e-20), depths, T0, want_volume=True)
    for r in (rc, rb):
        assert np.array_equal(r["poses"][..., 0], r0["poses"][..., 0])
        assert np.array_equal(r["F"][:, 0], r0["F"][:, 0])
        assert np.array_equal(r["W"][:, 0], r0["W"][:, 0])
        assert np.array_equal(r["stats"][:, [0, 1, 3, 4, 5]], r0["stats"][:, [0, 1, 3, 4, 5]])
