"""GPU: several independent sequences of uneven size advanced together (one
stream per instance, one frame each per round) give, per instance, exactly
the results of that instance run alone: the per-context arithmetic does not
depend on what runs beside it.  Also the fused 16-direction + 4x4 Hessian
shape against the shapes it contains."""
import numpy as np
import pytest

import scenegen as sg
from gpu_util import log, relerr, torch_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_02187_amd import multi as M  # noqa: E402
from paper_2405_02187_amd import xslam as X  # noqa: E402


def test_batch_equals_instances_run_alone():
    presets = sg.instance_presets(24)
    # a spread of shapes: both image sizes, several volumes, D from 1 to 6,
    # one with the depth-noise direction (needs its tangent frames)
    pick = [0, 1, 2, 3, 7, 9, 15, 21]
    insts = M.make_instances([presets[i] for i in pick], frame_cap=10)
    res = M.run_batch(insts, n_streams=4)
    log("batch of", len(insts), "instances:", res["value"], "frames*dirs/s, latency", res["latency_ms"])
    assert res["latency_ms"]["p50"] > 0
    for inst, sb in zip(insts, res["slams"]):
        sa, _ = M.run_alone(inst)
        Pa, Pb = sa.get(X.F_POSES), sb.get(X.F_POSES)
        Ca, Cb = sa.get(X.F_COUNTERS), sb.get(X.F_COUNTERS)
        log("instance", inst["preset"]["seed"], "dirs", inst["preset"]["dirs"], "frames", inst["n"],
            "lost", int(Ca[:, 0].sum()))
        assert np.array_equal(Pa, Pb)
        assert np.array_equal(Ca, Cb)
        sa.close()
        sb.close()


def test_fused_16_directions_and_4x4_hessian_shape():
    """One launch per stage carrying 16 first-order and 10 second-order parts
    (the Hessian over the first four directions) equals the 16-direction and
    the 4x4-Hessian shapes run separately: real parts and every part bit for
    bit up to the FP32 rounding of the shared reductions."""
    p = sg.preset("c0")
    seq = sg.make_sequence(p, n_frames=5)
    depths, tans = seq.depths_and_tangents()
    depths, tans = depths.astype(np.float32), tans.astype(np.float32)
    h = 2.0 ** -16
    params = list(sg.PARAMS16)
    hess = [X.P_TRUNC, X.P_WCAP, X.P_FX, X.P_DGATE]
    order = hess + [q for q in params if q not in hess]

    def run(dirs, q):
        cfg = X.config_from_preset(p, prec=X.C64, max_frames=len(depths))
        slam = X.Slam(cfg, X.Perturbation([(d, h) for d in dirs], q), seq.poses_gt[0])
        dev = torch_dev(depths, np.float32)
        ddev = torch_dev(tans, np.float32) if X.P_DEPTH in dirs else None
        for k in range(len(depths)):
            slam.step(dev[k], None if ddev is None else ddev[k])
        P, F = slam.get(X.F_POSES), slam.get(X.F_TSDF)
        slam.close()
        return P, F

    Pf, Ff = run(order, 4)
    P16, F16 = run(order, 0)
    P44, F44 = run(hess, 4)
    assert np.array_equal(Pf[:, 0], P16[:, 0]) and np.array_equal(Pf[:, 0], P44[:, 0])
    e1 = relerr(Pf[:, 1:17], P16[:, 1:17])
    e2 = relerr(Pf[:, 17:], P44[:, 5:])
    ef = relerr(Ff[1:17], F16[1:17])
    log("fused 16+10 vs separate: first order", e1, "second order", e2, "F first order", ef)
    assert e1 <= 1e-5 and e2 <= 1e-5 and ef <= 1e-5


def test_frame_graph_equals_eager_launches():
    """The tracked frame replayed as a captured graph (a context on a created
    stream) against the same frames launched kernel by kernel (the legacy null
    stream, which cannot be captured): poses, counters and the volume equal
    bit for bit (FP32, 2 directions, 12 frames of the 128^3 sequence)."""
    p = sg.preset("c0")
    n = 12
    seq = sg.make_sequence(p, n_frames=n)
    depths = seq.depths().astype(np.float32)

    def run(stream):
        with torch.cuda.stream(stream):
            cfg = X.config_from_preset(p, prec=X.C64, max_frames=n)
            slam = X.Slam(cfg, X.Perturbation([(X.P_PHI_X, 2.0 ** -20), (X.P_TRUNC, 2.0 ** -20)]),
                          seq.poses_gt[0])
            dev = torch.from_numpy(depths).cuda()
            for k in range(n):
                slam.step(dev[k])
            graph = slam.frame_graph()
            out = slam.get(X.F_POSES), slam.get(X.F_COUNTERS), slam.get(X.F_TSDF), graph
            slam.close()
        torch.cuda.synchronize()
        return out

    assert torch.cuda.default_stream().cuda_stream == 0
    Pe, Ce, Fe, ge = run(torch.cuda.default_stream())
    s = torch.cuda.Stream()
    assert s.cuda_stream != 0
    Pg, Cg, Fg, gg = run(s)
    assert not ge and gg
    log("frame graph vs eager: lost", int(Cg[:, 0].sum()), "hits", Cg[:, 2].tolist()[:4])
    assert np.array_equal(Pe, Pg)
    assert np.array_equal(Ce, Cg)
    assert np.array_equal(Fe, Fg)
