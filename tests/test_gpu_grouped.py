"""GPU: several independent sequences stepped by grouped launches (one grid
per stage for every context of a shape, each context's descriptor and work
items) give, per context, exactly the results of that context run alone,
also where a group holds one context; one FP64 member checked against the oracle; the batch's refusals."""
import ctypes as C

import numpy as np
import pytest

import oracle as O
import scenegen as sg
from gpu_util import gpu_pose_to_oracle, log, relerr, torch_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_02187_amd import multi as M  # noqa: E402
from paper_2405_02187_amd import xslam as X  # noqa: E402


def _instances():
    """Three shapes: five 2-direction contexts (both image sizes, 256^3 to
    384^3 at 1 and 2 cm, one with fewer ICP iterations), two 1-direction
    contexts, two 6-direction contexts perturbing the depth (their tangent
    frames are copied too); uneven lengths."""
    pr = sg.instance_presets(24)
    picks = [(4, 10), (10, 7), (12, 10), (16, 5), (21, 9), (9, 8), (15, 10), (1, 6), (7, 10)]
    presets = []
    for i, n in picks:
        p = dict(pr[i])
        p["n_frames"] = n
        if i == 10:
            p["icp"] = dict(p["icp"], iters=(6, 3, 2))
        presets.append(p)
    return M.make_instances(presets)


@pytest.mark.parametrize("persist", [0, 512])
def test_grouped_batch_equals_instances_run_alone(persist):
    insts = _instances()
    res = M.run_batch(insts, grouped=True, persist=persist)
    log("grouped batch, persist", persist, ":", res["value"], "frames*dirs/s on", res["streams"], "streams, latency",
        res["latency_ms"])
    assert res["latency_ms"]["p50"] > 0
    for inst, sb in zip(insts, res["slams"]):
        sa, _ = M.run_alone(inst)
        Pa, Pb = sa.get(X.F_POSES), sb.get(X.F_POSES)
        Ca, Cb = sa.get(X.F_COUNTERS), sb.get(X.F_COUNTERS)
        log("instance", inst["preset"]["seed"], "dirs", inst["preset"]["dirs"], "frames", inst["n"],
            "size", inst["preset"]["camera"]["width"], inst["preset"]["dim"], "lost", int(Ca[:, 0].sum()))
        assert Pa.shape[0] == inst["n"]
        assert np.array_equal(Pa, Pb)
        assert np.array_equal(Ca, Cb)
        if inst["preset"]["dim"] <= 256:
            assert np.array_equal(sa.get(X.F_TSDF), sb.get(X.F_TSDF))
            assert np.array_equal(sa.get(X.F_WEIGHT), sb.get(X.F_WEIGHT))
        sa.close()
        sb.close()


def test_grouped_single_member_groups_equal_instances_run_alone():
    """Groups of one context (a 1-direction and a 2-direction context of
    one size, each shape on a stream of its own): the same results as
    running each alone."""
    pr = sg.instance_presets(24)
    presets = []
    for i, n in ((9, 8), (4, 10)):
        p = dict(pr[i])
        p["n_frames"] = n
        presets.append(p)
    insts = M.make_instances(presets)
    assert len({M.shape_of(inst) for inst in insts}) == 2
    res = M.run_batch(insts, grouped=True)
    for inst, sb in zip(insts, res["slams"]):
        sa, _ = M.run_alone(inst)
        assert np.array_equal(sa.get(X.F_POSES), sb.get(X.F_POSES))
        assert np.array_equal(sa.get(X.F_COUNTERS), sb.get(X.F_COUNTERS))
        sa.close()
        sb.close()


def test_grouped_fp64_member_matches_oracle():
    """Three FP64 contexts of one shape (the 160x120 / 128^3 sequence from
    three initial poses, one pose direction) in one group: the first
    context's counts equal the oracle's and its poses (value and derivative)
    are within 1e-10."""
    p = sg.preset("c0")
    n = 8
    seq = sg.make_sequence(p, n_frames=n)
    d = seq.depths().astype(np.float64)
    T0 = seq.poses_gt[0]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        dev = torch_dev(d, np.float64)
        cfg = X.config_from_preset(p, prec=X.C128, max_frames=n)
        slams = []
        for k in range(3):
            T = T0.copy()
            T[:3, 3] += 0.002 * k
            slams.append(X.Slam(cfg, X.Perturbation([(X.P_RHO_Y, 1e-20)]), T))
        b = X.Batch(slams, grouped=True)
        for k in range(n):
            b.step([dev[k]] * 3)
        s.synchronize()
        P0 = slams[0].get(X.F_POSES)
        P = gpu_pose_to_oracle(P0)
        cnt = slams[0].get(X.F_COUNTERS)
        P2 = slams[2].get(X.F_POSES)
        b.close()
        for x in slams:
            x.close()
    ref = O.run_sequence(O.config(p), O.seed(1, O.P_RHO_Y, h=1e-20), d, T0)
    st = ref["stats"]
    assert np.array_equal(cnt[:, 0], st[:, 0].astype(int))
    assert np.array_equal(cnt[:, 1], st[:, 3].astype(int))
    assert np.array_equal(cnt[:, 2], st[:, 4].astype(int))
    assert np.array_equal(cnt[:, 3], st[:, 5].astype(int))
    e_re = relerr(P[..., 0], ref["poses"][..., 0])
    e_im = relerr(P[..., 1], ref["poses"][..., 1])
    log("grouped fp64 member vs oracle: pose", e_re, "derivative", e_im)
    assert e_re <= 1e-10 and e_im <= 1e-10
    assert P2.shape == P0.shape and not np.array_equal(P2[:, 0], P0[:, 0])   # the others tracked on their own


def test_grouped_batch_refusals():
    p = sg.preset("c0")
    T0 = sg.make_sequence(p, n_frames=1).poses_gt[0]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    cfg = X.config_from_preset(p, prec=X.C64, max_frames=4)
    with torch.cuda.stream(s1):
        a = X.Slam(cfg, X.Perturbation([(X.P_TRUNC, 2.0 ** -20)]), T0)
        surf = X.Slam(X.config_from_preset(p, prec=X.C64, max_frames=4, map=X.MAP_SURFEL),
                      X.Perturbation([(X.P_TRUNC, 2.0 ** -20)]), T0)
    with torch.cuda.stream(s2):
        b = X.Slam(cfg, X.Perturbation([(X.P_TRUNC, 2.0 ** -20)]), T0)
        c = X.Slam(cfg, X.Perturbation([(X.P_TRUNC, 2.0 ** -20), (X.P_FX, 2.0 ** -20)]), T0)
    L = X.lib()

    def create(slams, persist=0):
        arr = (C.c_void_p * len(slams))(*[x.h for x in slams])
        h = C.c_void_p()
        rc = L.xslam_batch_create_grouped(arr, len(slams), persist, C.byref(h))
        if rc == 0:
            L.xslam_batch_destroy(h)
        return rc

    assert create([a, b]) == 0                         # one shape on two streams: two groups
    assert create([a, c]) == 0                         # two shapes
    assert create([a], persist=12) == X.ERR_ARG        # not a multiple of 8
    assert create([a], persist=-8) == X.ERR_ARG
    assert create([a, surf]) == X.ERR_UNSUPPORTED
    assert "TSDF" in L.xslam_last_error(surf.h).decode()
    for x in (a, b, c, surf):
        x.close()
