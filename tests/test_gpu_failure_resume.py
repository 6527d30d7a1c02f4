"""GPU against the oracle on the failure paths, on constant velocity and on
the trajectory error, and checkpoint/resume of a sequence.

Every context here is created on a fresh stream, so its tracked frames replay
the captured frame graph (lost tracking is predicated on the device there).

* Failure paths (Sec. 4.1 ICP; readings: tracking is lost when fewer than 6
  correspondences remain or the 6x6 normal matrix has a non-positive pivot,
  and a lost frame keeps its initial pose and skips fusion): an all-zero
  depth frame, NaN / +-Inf / negative pixels in every frame, a scene that is a
  single plane (the normal matrix is rank 3), and a camera outside the volume
  looking away from it.  Per-frame lost flags and counts (fused voxels,
  raycast hits, ICP correspondences) equal the oracle's, poses and their
  derivative within 1e-10.
* Constant velocity (icp init 1): the same FP64 parity on the 20-frame 128^3
  sequence.
* Trajectory error (translational RMSE without alignment, Table 2's ATE):
  E and dE/dtheta from the library against the oracle's, 1e-10; and the
  zero-error case, where E has a kink and both give the one-sided derivative.
* Resume: 10 frames, checkpoint (get), a new context loaded with it (set),
  10 more frames equal 20 frames run straight through, bit for bit.
"""
import numpy as np
import pytest

import oracle as O
import scenegen as sg
from gpu_util import created_stream, gpu_pose_to_oracle, log, oracle_map_to_gpu, relerr, torch_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_02187_amd import xslam as X  # noqa: E402

H20 = 1e-20
NF = 6


def _run_both(p, depths, T0, param=O.P_TRUNC, init=0):
    """GPU FP64 (graph path) and oracle on the same depths -> (gpu counters,
    gpu poses (n,4,4,2), oracle result)."""
    n = len(depths)
    with created_stream():
        cfg = X.config_from_preset(p, prec=X.C128, max_frames=n, init=init)
        slam = X.Slam(cfg, X.Perturbation([(param, H20)]), T0)
        dev = torch_dev(depths, np.float64)
        for k in range(n):
            slam.step(dev[k])
        slam.sync()
        graph = slam.frame_graph()
        cnt = slam.get(X.F_COUNTERS)
        P = gpu_pose_to_oracle(slam.get(X.F_POSES))
        slam.close()
    ref = O.run_sequence(O.config(p, init=init), O.seed(1, param, h=H20), depths, T0)
    return cnt, P, ref, graph


def _assert_parity(cnt, P, ref, what):
    st = ref["stats"]
    log(what, "lost gpu", cnt[:, 0].tolist(), "oracle", st[:, 0].astype(int).tolist(),
        "fused", cnt[:, 1].tolist(), "hits", cnt[:, 2].tolist(), "corr", cnt[:, 3].tolist())
    assert np.array_equal(cnt[:, 0], st[:, 0].astype(int))
    assert np.array_equal(cnt[:, 1], st[:, 3].astype(int))
    assert np.array_equal(cnt[:, 2], st[:, 4].astype(int))
    assert np.array_equal(cnt[:, 3], st[:, 5].astype(int))
    e0 = relerr(P[..., 0], ref["poses"][..., 0])
    e1 = relerr(P[..., 1], ref["poses"][..., 1])
    log(what, "pose", e0, "derivative", e1)
    assert e0 <= 1e-10 and e1 <= 1e-10


def _c0(n=NF):
    p = sg.preset("c0")
    seq = sg.make_sequence(p, n_frames=n)
    return p, seq


def test_all_zero_depth_frame_is_lost():
    p, seq = _c0()
    d = seq.depths().astype(np.float64)
    d[3] = 0.0
    cnt, P, ref, graph = _run_both(p, d, seq.poses_gt[0])
    assert graph
    assert cnt[3, 0] == 1 and cnt[3, 1] == 0          # lost, nothing fused
    assert np.array_equal(P[3], P[2])                   # pose kept (initial estimate = previous pose)
    _assert_parity(cnt, P, ref, "zero depth")


def test_nan_inf_and_negative_pixels_are_invalid():
    p, seq = _c0()
    d = seq.depths().astype(np.float64)
    rng = np.random.default_rng(5)
    f = 0.001        # each kind; 0.4% of the pixels invalid in all
    for k in range(NF):
        m = rng.random(d[k].shape)
        d[k][m < f] = np.nan
        d[k][(m >= f) & (m < 2 * f)] = np.inf
        d[k][(m >= 2 * f) & (m < 3 * f)] = -np.inf
        d[k][(m >= 3 * f) & (m < 4 * f)] = -0.5
    cnt, P, ref, graph = _run_both(p, d, seq.poses_gt[0])
    assert cnt[1:, 0].sum() == 0                        # still tracks
    assert np.isfinite(P).all()
    _assert_parity(cnt, P, ref, "nan/inf")


def test_single_plane_normal_matrix_is_rank_deficient_and_lost():
    """Analytic model maps of a single plane (every model normal the same) and
    the noise-free depth of that plane: the translations within the plane and
    the rotation about its normal leave every residual unchanged, so the 6x6
    normal matrix has rank 3 and a pivot at rounding level; both sides report
    tracking lost and keep the pose."""
    p = sg.preset("c0")
    cam = p["camera"]
    W, H = cam["width"], cam["height"]
    kc = {k: cam[k] for k in ("fx", "fy", "cx", "cy")}
    sc = sg.make_scene(p["seed"], p["L"])
    plane = sg.Scene(L=sc.L, floor_y=sc.floor_y, spheres=np.zeros((0, 4)), boxes=np.zeros((0, 6)))
    T = sg.look_at((0.3, 0.2, -0.9), (0.0, sc.floor_y, 0.2))
    z, Pw, Nw = sg.render_maps(plane, T, W, H, **kc)
    assert (z > 0).mean() > 0.9
    s = O.seed(1, O.P_TRUNC, h=H20)
    model = dict(V=O.lift(Pw, s), N=O.lift(Nw, s), Z=z, valid=(z > 0).astype(np.uint8))
    Tl = O.lift(T, s)
    Tr, lost_r, cnt_r, _ = O.track(O.config(p), s, z, None, model, Tl, Tl)
    with created_stream():
        cfg = X.config_from_preset(p, prec=X.C128, max_frames=4)
        slam = X.Slam(cfg, X.Perturbation([(X.P_TRUNC, H20)]), T)
        slam.set(X.F_VMAP, oracle_map_to_gpu(model["V"]))
        slam.set(X.F_NMAP, oracle_map_to_gpu(model["N"]))
        slam.set(X.F_ZMAP, z.reshape(-1))
        slam.set(X.F_MVALID, model["valid"].reshape(-1))
        rc, pose = slam.track(torch_dev(z, np.float64))
        slam.close()
    log("single plane: oracle lost", lost_r, "correspondences", cnt_r, "gpu rc", rc)
    assert lost_r == 1 and rc == 1                      # XSLAM_WARN_TRACK_LOST
    Pg = np.moveaxis(pose.reshape(2, 4, 4), 0, -1)
    assert np.array_equal(Pg[..., 0], T)
    assert np.array_equal(Tr[..., 0], T)


def test_camera_outside_the_volume_looking_away():
    p = sg.preset("c0")
    sc = sg.make_scene(p["seed"], p["L"])
    eye = np.array([0.0, 0.0, 3.0])                     # cube half-size 1.28 m
    poses = np.stack([sg.look_at(eye + [0.01 * k, 0, 0], eye + [0.01 * k, -0.5, 3.0]) for k in range(NF)])
    seq = sg.Sequence(scene=sc, poses_gt=poses, camera=p["camera"], seed=p["seed"], depth_dtype=np.float64)
    d = seq.depths()
    assert (d > 0).mean() > 0.2                         # the floor is seen, outside the volume
    cnt, P, ref, graph = _run_both(p, d, poses[0])
    assert cnt[:, 1].sum() == 0 and cnt[:, 2].sum() == 0   # nothing fused, nothing hit
    assert cnt[1:, 0].min() == 1
    _assert_parity(cnt, P, ref, "outside")


def test_constant_velocity_sequence_matches_oracle():
    p, seq = _c0(20)
    d = seq.depths().astype(np.float64)
    cnt, P, ref, graph = _run_both(p, d, seq.poses_gt[0], param=O.P_RHO_X, init=1)
    assert graph
    _assert_parity(cnt, P, ref, "constant velocity")
    # it differs from the previous-pose start from frame 2 on
    ref0 = O.run_sequence(O.config(p), O.seed(1, O.P_RHO_X, h=H20), d, seq.poses_gt[0])
    assert np.array_equal(ref0["poses"][:2], ref["poses"][:2])
    assert not np.array_equal(ref0["poses"][2:], ref["poses"][2:])


@pytest.mark.parametrize("param", [O.P_TRUNC, O.P_PHI_Y])
def test_trajectory_error_matches_oracle(param):
    p, seq = _c0(20)
    d = seq.depths().astype(np.float64)
    gt = seq.poses_gt
    s = O.seed(1, param, h=H20)
    with created_stream():
        cfg = X.config_from_preset(p, prec=X.C128, max_frames=len(d))
        slam = X.Slam(cfg, X.Perturbation([(param, H20)]), gt[0])
        dev = torch_dev(d, np.float64)
        for k in range(len(d)):
            slam.step(dev[k])
        E = slam.traj_err(gt)
        P = gpu_pose_to_oracle(slam.get(X.F_POSES))
        # the zero-error case: the reference is the run's own real trajectory
        E0 = slam.traj_err(P[..., 0])
        slam.close()
    ref = O.run_sequence(O.config(p), s, d, gt[0])
    Er = O.traj_err(s, ref["poses"], gt)
    log("traj err gpu", E, "oracle", Er)
    assert relerr(E[0], Er[0]) <= 1e-10 and relerr(E[1], Er[1]) <= 1e-10
    Er0 = O.traj_err(s, ref["poses"], ref["poses"][..., 0])
    log("zero-error case gpu", E0, "oracle", Er0)
    assert E0[0] == 0.0 and Er0[0] == 0.0
    assert np.isfinite(E0).all() and E0[1] > 0
    assert relerr(E0[1], Er0[1]) <= 1e-10


@pytest.mark.parametrize("init", [0, 1])
def test_resume_from_checkpoint_is_bit_exact(init):
    p, seq = _c0(20)
    d = seq.depths().astype(np.float64)
    T0 = seq.poses_gt[0]
    pert = X.Perturbation([(X.P_RHO_Y, H20)])
    with created_stream():
        cfg = X.config_from_preset(p, prec=X.C128, max_frames=20, init=init)
        dev = torch_dev(d, np.float64)
        a = X.Slam(cfg, pert, T0)
        for k in range(20):
            a.step(dev[k])
        b = X.Slam(cfg, pert, T0)
        for k in range(10):
            b.step(dev[k])
        ck = b.save_state()
        b.close()
        c = X.Slam(cfg, pert, T0)
        c.load_state(ck)
        for k in range(10, 20):
            c.step(dev[k])
        assert c.frame_graph()
        for f in (X.F_POSES, X.F_COUNTERS, X.F_TSDF, X.F_WEIGHT, X.F_VMAP, X.F_NMAP, X.F_MVALID, X.F_POSE):
            ga, gc = a.get(f), c.get(f)
            assert np.array_equal(ga, gc), f
        assert np.array_equal(a.traj_err(seq.poses_gt), c.traj_err(seq.poses_gt))
        log("resume init", init, "bit-exact over", a.frame(), "frames")
        a.close()
        c.close()
