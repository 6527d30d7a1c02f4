"""GPU Newton ICP (Sec. 4.1, the second-order ICP step) against the oracle,
and the optimiser comparison of Sec. 5.1 (Fig. 3).

* ``xslam_icp_energy``: E = sum r^2 of one pass with its gradient and
  Hessian in the pose increment (the library: six hyper-dual directions and
  21 pairs per pixel; the oracle: 6 complex-step and 21 bicomplex runs of the
  same pass), correspondences held fixed or through the association, at a
  pose away from the solution, levels 0-2: count equal, E, g and H within
  1e-10 (FP64); the same at the benchmark's size (640x480, 512^3), level 0,
  through the association.
* Tracking with the Newton solvers (correspondences held fixed per pass, or
  differentiated through the association) on the 128^3 sequence (FP64, no
  directions): per-frame counts equal, poses within 1e-10 of the oracle.
* Gradient descent, nonlinear CG and Newton from the same start on the same
  objective (the library evaluates it): traces logged; Newton converges.
"""
import numpy as np
import pytest

import oracle as O
import scenegen as sg
from gpu_util import created_stream, log, oracle_map_to_gpu, relerr, torch_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_02187_amd import icp_methods as IM  # noqa: E402
from paper_2405_02187_amd import xslam as X  # noqa: E402


def _set_model(slam, V, N, Z, valid):
    slam.set(X.F_VMAP, oracle_map_to_gpu(V))
    slam.set(X.F_NMAP, oracle_map_to_gpu(N))
    slam.set(X.F_ZMAP, np.ascontiguousarray(Z, np.float64).reshape(-1))
    slam.set(X.F_MVALID, np.ascontiguousarray(valid, np.uint8).reshape(-1))


@pytest.mark.parametrize("through", [False, True])
def test_icp_energy_matches_oracle(through):
    p = sg.preset("c0")
    seq = sg.make_sequence(p, n_frames=4)
    d = seq.depths().astype(np.float64)
    T0 = seq.poses_gt[0]
    s0 = O.seed(0)
    c = O.config(p)
    r = O.run_sequence(c, s0, d[:3], T0, want_volume=True)
    Tprev = r["poses"][2][..., 0]
    model = O.raycast(c, s0, r["F"], r["W"], Tprev[..., None])
    meas = O.measure(c, s0, d[3])
    Tj = IM.se3_exp([0.006, -0.004, 0.003, 0.012, -0.008, 0.01]) @ Tprev
    with created_stream():
        cfg = X.config_from_preset(p, prec=X.C128, max_frames=8)
        slam = X.Slam(cfg, X.Perturbation([]), T0)
        _set_model(slam, model["V"], model["N"], model["Z"], model["valid"])
        slam.set(X.F_PREV_POSE, Tprev[None])
        slam.measure(torch_dev(d[3], np.float64))
        slam.set(X.F_POSE, Tj[None])
        for l in range(3):
            sub = 2 ** l
            mod_l = {k: v[::sub, ::sub] for k, v in model.items()}
            E, g, H, cnt = slam.icp_energy(l, through)
            Er, gr, Hr, cr = O.icp_energy(c, l, meas[l], mod_l, Tprev, Tj, through=through)
            log("through", through, "level", l, "count", cnt, cr, "E", E, Er, "g err", relerr(g, gr), "H err",
                relerr(H, Hr))
            assert cnt == cr
            assert relerr(E, Er) <= 1e-10
            assert relerr(g, gr) <= 1e-10
            assert relerr(H, Hr) <= 1e-10
        slam.close()


def test_icp_energy_fullsize_matches_oracle():
    """The Newton objective at the benchmark's size (640x480 against the model
    maps raycast from the oracle's 512^3 volume after two frames), with the
    correspondences differentiated through the association, level 0: count
    equal, E, g and H within 1e-10 (FP64)."""
    p = sg.preset("c1")
    seq = sg.make_sequence(p, n_frames=3)
    d = seq.depths().astype(np.float64)
    T0 = seq.poses_gt[0]
    s0 = O.seed(0)
    c = O.config(p)
    r = O.run_sequence(c, s0, d[:2], T0, want_volume=True)
    Tprev = r["poses"][1][..., 0]
    model = O.raycast(c, s0, r["F"], r["W"], Tprev[..., None])
    meas = O.measure(c, s0, d[2])
    Tj = IM.se3_exp([0.004, -0.003, 0.002, 0.008, -0.005, 0.006]) @ Tprev
    with created_stream():
        cfg = X.config_from_preset(p, prec=X.C128, max_frames=4)
        slam = X.Slam(cfg, X.Perturbation([]), T0)
        _set_model(slam, model["V"], model["N"], model["Z"], model["valid"])
        slam.set(X.F_PREV_POSE, Tprev[None])
        slam.measure(torch_dev(d[2], np.float64))
        slam.set(X.F_POSE, Tj[None])
        E, g, H, cnt = slam.icp_energy(0, True)
        slam.close()
    Er, gr, Hr, cr = O.icp_energy(c, 0, meas[0], model, Tprev, Tj, through=True)
    log("full-size Newton objective: count", cnt, cr, "E", E, Er, "g err", relerr(g, gr), "H err", relerr(H, Hr))
    assert cnt == cr > 100000
    assert relerr(E, Er) <= 1e-10
    assert relerr(g, gr) <= 1e-10
    assert relerr(H, Hr) <= 1e-10


@pytest.mark.parametrize("solver", [1, 2])
def test_newton_tracking_sequence_matches_oracle(solver):
    p = sg.preset("c0")
    n = 4
    seq = sg.make_sequence(p, n_frames=n)
    d = seq.depths().astype(np.float64)
    T0 = seq.poses_gt[0]
    iters = (4, 2, 2)
    with created_stream():
        cfg = X.config_from_preset(p, prec=X.C128, max_frames=n, solver=solver, iters=iters)
        slam = X.Slam(cfg, X.Perturbation([]), T0)
        dev = torch_dev(d, np.float64)
        for k in range(n):
            slam.step(dev[k])
        cnt = slam.get(X.F_COUNTERS)
        P = slam.get(X.F_POSES)[:, 0]
        assert slam.frame_graph()
        slam.close()
    ref = O.run_sequence(O.config(p, solver=solver, iters=iters), O.seed(0), d, T0)
    st = ref["stats"]
    log("newton counts gpu", cnt[:, :4].tolist(), "oracle", st[:, [0, 3, 4, 5]].tolist(),
        "gauss-newton fall-backs", cnt[:, 34].tolist())
    assert np.array_equal(cnt[:, 0], st[:, 0].astype(int))
    assert np.array_equal(cnt[:, 1], st[:, 3].astype(int))
    assert np.array_equal(cnt[:, 2], st[:, 4].astype(int))
    assert np.array_equal(cnt[:, 3], st[:, 5].astype(int))
    e = relerr(P, ref["poses"][..., 0])
    log("newton tracking (solver", solver, ") fp64 vs oracle: pose", e)
    assert e <= 1e-10


def test_optimiser_comparison_runs_and_newton_converges():
    p = sg.preset("c0")
    cam = p["camera"]
    W, H = cam["width"], cam["height"]
    kc = {k: cam[k] for k in ("fx", "fy", "cx", "cy")}
    sc = sg.make_scene(p["seed"], p["L"])
    T_ref = sg.circle_trajectory(1, 1.5, 0.0, 2.0)[0]
    rng = np.random.default_rng(11)
    ax = rng.normal(size=3)
    ax /= np.linalg.norm(ax)
    tr = rng.normal(size=3)
    tr /= np.linalg.norm(tr)
    xi = np.concatenate([np.radians(3.0) * ax, 0.04 * tr])      # a random 3 degree / 4 cm transform
    T_true = IM.se3_exp(xi) @ T_ref
    z_src = sg.render_depth(sc, T_true, W, H, **kc)
    zm, Pm, Nm = sg.render_maps(sc, T_ref, W, H, **kc)
    with created_stream():
        cfg = X.config_from_preset(p, prec=X.C128, max_frames=4)
        slam = X.Slam(cfg, X.Perturbation([]), T_ref)
        _set_model(slam, Pm[..., None], Nm[..., None], zm, zm > 0)
        slam.set(X.F_PREV_POSE, T_ref[None])
        slam.measure(torch_dev(z_src, np.float64))
        res = IM.run(slam, 0, T_ref, T_true, iters=15)
        slam.close()
    for m, r in res.items():
        tr_ = r["trace"]
        log(m, "evaluations", r["evaluations"], "t err", [round(x["t_err_m"], 6) for x in tr_][:16])
        assert all(np.isfinite(x["E"]) for x in tr_)
    newton, gd = res["newton"]["trace"], res["gd"]["trace"]
    # the objective's minimum sits a few mm from the true pose (silhouettes,
    # the filtered source depth); Newton reaches it and stays
    assert newton[-1]["t_err_m"] < 5e-3
    # converged: the last iterates stay within 0.1 mm of each other
    assert abs(newton[-1]["t_err_m"] - newton[-3]["t_err_m"]) < 1e-4
    assert newton[-1]["E"] <= gd[-1]["E"] * (1 + 1e-9)
