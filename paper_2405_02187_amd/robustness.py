"""Tracking robustness against the frame step (Sec. 5.1, the comparison of
X-KF with the original KF at frame steps 1, 2 and 3): the sequence is
subsampled to every s-th frame, so the camera moves s times farther between
tracked frames, and the translational RMSE of the trajectory (no alignment)
is reported for each pose-update form of the ICP:

* ``exp``: the exact SE(3) exponential T <- exp(delta) T (this library's
  default; the paper's X-KF update),
* ``small_angle``: the linearised increment of eq. icp_approx, the original
  KF's form (rotation re-orthonormalised after the update),
* ``newton``: the exact exponential with Newton steps (the complex-step
  Hessian of the pass's objective, correspondences held fixed), the paper's
  second-order ICP,
* ``newton_assoc``: Newton steps on the objective differentiated through the
  projective association.

The paper measures this on ICL-NUIM lr kt2 (not available here); the seeded
synthetic 640x480 / 512^3 spline sequence stands in for it.
"""
from __future__ import annotations

import numpy as np

from . import xslam as X

# form name -> (icp.update, icp.solver)
FORMS = {"exp": (0, 0), "small_angle": (1, 0), "newton": (0, 1), "newton_assoc": (0, 2)}


def run(preset: dict, depths: np.ndarray, poses_gt: np.ndarray, steps=(1, 2, 3), n_frames: int = 60,
        prec=X.C64, device="cuda:0", forms=FORMS) -> list:
    """depths/poses_gt: the full-rate sequence (at least 1 + (n_frames-1) *
    max(steps) frames).  -> list of dict(step, form, ate_m, max_err_m,
    lost_frames, iters_to_converge_mean)."""
    import torch
    out = []
    dt = np.float32 if prec == X.C64 else np.float64
    for s in steps:
        idx = np.arange(n_frames) * s
        assert idx[-1] < len(depths), "sequence too short for this frame step"
        dev = torch.from_numpy(np.ascontiguousarray(depths[idx], dtype=dt)).to(device)
        gt = poses_gt[idx]
        for name, (upd, solver) in forms.items():
            cfg = X.config_from_preset(preset, prec=prec, max_frames=n_frames, update=upd, solver=solver)
            slam = X.Slam(cfg, X.Perturbation([]), gt[0], device=device)
            for k in range(n_frames):
                slam.step(dev[k])
            ate = float(slam.traj_err(gt)[0])
            P = slam.get(X.F_POSES)[:, 0]
            err = np.linalg.norm(P[:, :3, 3] - gt[:, :3, 3], axis=1)
            cnt = slam.get(X.F_COUNTERS)
            conv = cnt[1:, 32]
            slam.close()
            out.append(dict(step=int(s), form=name, frames=n_frames, ate_m=ate, max_err_m=float(err.max()),
                            lost_frames=int(cnt[:, 0].sum()),
                            first_converged_pass_mean=float(conv[conv > 0].mean()) if (conv > 0).any() else None))
        del dev
    return out
