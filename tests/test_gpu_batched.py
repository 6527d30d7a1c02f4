"""GPU: batched directions and hyper-dual second derivatives.

* Several directions sharing one real part in one launch give, per direction,
  the same tangent as a single-direction run (the real part is the same and a
  first-order part only meets real parts and itself).
* The hyper-dual Hessian parts (i1*i2 of eq. csfd_hessian) match the bicomplex
  oracle (Sec. 3, eqs. multi_complex / mc_taylor) within 1e-10 in FP64, and a
  fused Hessian shape agrees with the smaller shapes it contains.
"""
import numpy as np
import pytest

import oracle as O
import scenegen as sg
from gpu_util import gpu_pose_to_oracle, log, relerr, torch_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_02187_amd import xslam as X  # noqa: E402

H20 = 1e-20


def run(p, depths, T0, prec, dirs, q=0, n=None):
    n = len(depths) if n is None else n
    cfg = X.config_from_preset(p, prec=prec, max_frames=n)
    slam = X.Slam(cfg, X.Perturbation(dirs, q), T0)
    dev = torch_dev(depths[:n], np.float64 if prec == X.C128 else np.float32)
    for k in range(n):
        slam.step(dev[k])
    P = slam.get(X.F_POSES)
    F = slam.get(X.F_TSDF)
    slam.close()
    return P, F


def test_batched_directions_equal_single_runs_fp64():
    p = sg.preset("c0")
    seq = sg.make_sequence(p, n_frames=8)
    depths = seq.depths()
    T0 = seq.poses_gt[0]
    params = [X.P_PHI_X, X.P_PHI_Y, X.P_RHO_Z, X.P_TRUNC, X.P_FX, X.P_CY]
    P6, F6 = run(p, depths, T0, X.C128, [(q, H20) for q in params])
    for d, q in enumerate(params):
        P1, F1 = run(p, depths, T0, X.C128, [(q, H20)])
        assert np.array_equal(P6[:, 0], P1[:, 0]), d
        e = relerr(P6[:, 1 + d], P1[:, 1])
        ef = relerr(F6[1 + d], F1[1])
        log("batched vs single", q, e, ef)
        assert e <= 1e-13 and ef <= 1e-13


def test_batched_directions_match_oracle_fp64():
    """Six directions in one FP64 launch against the oracle's complex-step run
    of each direction (its own seed), 4 frames of the 128^3 sequence: real
    parts of the poses within 1e-12, every tangent within 1e-10, the volume's
    tangent planes within 1e-10."""
    p = sg.preset("c0")
    n = 4
    seq = sg.make_sequence(p, n_frames=n)
    depths = seq.depths()
    T0 = seq.poses_gt[0]
    params = [X.P_PHI_X, X.P_PHI_Y, X.P_RHO_Z, X.P_TRUNC, X.P_FX, X.P_CY]
    P6, F6 = run(p, depths, T0, X.C128, [(q, H20) for q in params])
    c = O.config(p)
    d64 = depths[:n].astype(np.float64)
    for d, q in enumerate(params):
        r = O.run_sequence(c, O.seed(1, q, h=H20), d64, T0, want_volume=True)
        Pr = np.moveaxis(r["poses"], -1, 1)                     # (n, 2, 4, 4)
        e_re = relerr(P6[:, 0], Pr[:, 0])
        e_tan = relerr(P6[:, 1 + d], Pr[:, 1])
        e_f = relerr(F6[1 + d], r["F"][:, 1])
        log("batched direction", q, "vs oracle: pose", e_re, "tangent", e_tan, "F tangent", e_f)
        assert e_re <= 1e-12 and e_tan <= 1e-10 and e_f <= 1e-10


def test_batched_16_directions_fp32_equal_single_runs():
    p = sg.preset("c0")
    seq = sg.make_sequence(p, n_frames=6)
    depths = seq.depths().astype(np.float32)
    T0 = seq.poses_gt[0]
    params = [X.P_PHI_X, X.P_PHI_Y, X.P_PHI_Z, X.P_RHO_X, X.P_RHO_Y, X.P_RHO_Z, X.P_TRUNC, X.P_WCAP,
              X.P_DGATE, X.P_AGATE, X.P_ICPW0, X.P_ICPW1, X.P_ICPW2, X.P_FX, X.P_FY, X.P_CX]
    h = 2.0 ** -20
    P16, _ = run(p, depths, T0, X.C64, [(q, h) for q in params])
    for d in (0, 6, 13):
        P1, _ = run(p, depths, T0, X.C64, [(params[d], h)])
        assert np.array_equal(P16[:, 0], P1[:, 0])
        e = relerr(P16[:, 1 + d], P1[:, 1])
        log("16-batched vs single", params[d], e)
        assert e <= 1e-5
    # hard gates: exactly zero derivative
    for d in (8, 9):
        assert np.all(P16[:, 1 + d] == 0.0)


@pytest.mark.parametrize("pa,pb", [(X.P_TRUNC, X.P_FX), (X.P_TRUNC, X.P_RHO_X)])
def test_hyperdual_hessian_matches_bicomplex_oracle_fp64(pa, pb):
    p = sg.preset("c0")
    n = 8
    seq = sg.make_sequence(p, n_frames=n)
    depths = seq.depths()
    T0 = seq.poses_gt[0]
    P, _ = run(p, depths, T0, X.C128, [(pa, H20), (pb, H20)], q=2)   # comps: re, a, b, aa, ab, bb
    c = O.config(p)
    for comp, (oa, ob) in [(3, (pa, pa)), (4, (pa, pb)), (5, (pb, pb))]:
        ref = O.run_sequence(c, O.seed(2, oa, ob, H20), depths, T0)["poses"]
        e = relerr(P[:, comp], ref[..., 3])
        log("hessian", oa, ob, "rel err", e)
        assert e <= 1e-10
    for comp, q in [(1, pa), (2, pb)]:
        ref = O.run_sequence(c, O.seed(1, q, h=H20), depths, T0)["poses"]
        assert relerr(P[:, comp], ref[..., 1]) <= 1e-10


def test_fused_hessian_shape_contains_small_shape_fp32():
    p = sg.preset("c0")
    seq = sg.make_sequence(p, n_frames=5)
    depths = seq.depths().astype(np.float32)
    T0 = seq.poses_gt[0]
    h = 2.0 ** -16
    params = [X.P_TRUNC, X.P_WCAP, X.P_FX, X.P_DGATE]
    P4, _ = run(p, depths, T0, X.C64, [(q, h) for q in params], q=4)   # 1 + 4 + 10 comps
    P2, _ = run(p, depths, T0, X.C64, [(params[0], h), (params[2], h)], q=2)
    assert np.array_equal(P4[:, 0], P2[:, 0])
    # pairs over (0..3): (0,0)=5, (0,1)=6, (0,2)=7, ...; small shape: (0,0)=3, (0,1)=4, (1,1)=5
    assert relerr(P4[:, 5], P2[:, 3]) <= 1e-5
    assert relerr(P4[:, 7], P2[:, 4]) <= 1e-5
    # d2/dfx2: pairs index of (2,2) in the 4x4 upper triangle is 5+7=12
    assert relerr(P4[:, 12], P2[:, 5]) <= 1e-5


@pytest.mark.parametrize("nframes", [1, 2])
def test_hyperdual_volume_and_pose_first_frames_fp64(nframes):
    """Second-order parts of the TSDF (after fusion) and of the first tracked
    pose against the bicomplex oracle, pair by pair."""
    p = sg.preset("c0")
    seq = sg.make_sequence(p, n_frames=nframes)
    depths = seq.depths()
    T0 = seq.poses_gt[0]
    pa, pb = X.P_TRUNC, X.P_FX
    P, F = run(p, depths, T0, X.C128, [(pa, H20), (pb, H20)], q=2)
    c = O.config(p)
    for comp, (oa, ob) in [(3, (pa, pa)), (4, (pa, pb)), (5, (pb, pb))]:
        ref = O.run_sequence(c, O.seed(2, oa, ob, H20), depths, T0, want_volume=True)
        eF = relerr(F[comp], ref["F"][:, 3])
        eP = relerr(P[:, comp], ref["poses"][..., 3])
        log("frames", nframes, "pair", oa, ob, "F rel err", eF, "pose rel err", eP)
        assert eF <= 1e-10 and eP <= 1e-10
