"""FP32-complex against FP64-complex, one frame step from the same state.

Over a long sequence the FP32 and FP64 trajectories drift apart the way any
two runs of a thresholded method do (a flipped gate moves the least-squares
solution, and the next frames start from there).  To measure the arithmetic
of one frame step instead, an FP64 context is run to frame k, its state
(TSDF with its tangent, weights, model maps of the previous frame, pose) is
rounded into an FP32 context, and both step frame k on the same input.
"""
from __future__ import annotations

import numpy as np

from . import xslam as X


def _rel(a, b):
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


def _copy_state(src, dst, scale):
    """The state a tracked frame step reads, from src into dst, tangents x scale."""
    F, Wt = src.get(X.F_TSDF), src.get(X.F_WEIGHT)
    F[1:] *= scale
    Wt[1:] *= scale
    dst.set(X.F_TSDF, F)
    dst.set(X.F_WEIGHT, Wt)
    del F, Wt
    V, N = src.get(X.F_VMAP), src.get(X.F_NMAP)
    V[:, 1:] *= scale
    N[:, 1:] *= scale
    dst.set(X.F_VMAP, V)
    dst.set(X.F_NMAP, N)
    dst.set(X.F_ZMAP, src.get(X.F_ZMAP))
    dst.set(X.F_MVALID, src.get(X.F_MVALID))
    P = src.get(X.F_POSE)
    P[1:] *= scale
    dst.set(X.F_POSE, P)
    dst.set_frame(src.frame())


def one_step_errors(preset: dict, depths32: np.ndarray, T0: np.ndarray, ks, param: int = X.P_PHI_X,
                    h64: float = 1e-20, h32: float = 2.0 ** -20, jitter: float = 6e-8, device="cuda:0"):
    """depths32: (n, H, W) float32 frames (the FP64 context gets them widened
    exactly).  -> list of dict(frame, pose_rel_err, grad_rel_err,
    pose_spread, grad_spread) for every frame k in ks (1 <= k < n); the
    spreads are what the FP64 step itself moves when its input depth is
    jittered at FP32 resolution (relative ``jitter``), from the same state:
    the conditioning that any rounding of the step meets."""
    import torch
    ks = sorted(int(k) for k in ks)
    n = int(ks[-1]) + 1
    cfg64 = X.config_from_preset(preset, prec=X.C128, max_frames=n)
    cfg32 = X.config_from_preset(preset, prec=X.C64, max_frames=n)
    a = X.Slam(cfg64, X.Perturbation([(param, h64)]), T0, device=device)
    d64 = torch.from_numpy(depths32[:n].astype(np.float64)).to(device)
    d32 = torch.from_numpy(np.ascontiguousarray(depths32[:n], dtype=np.float32)).to(device)
    s = h32 / h64                       # tangent planes hold h times the derivative
    rng = np.random.default_rng(0)
    out, done = [], 0
    for k in ks:
        for j in range(done, k):
            a.step(d64[j])
        b = X.Slam(cfg32, X.Perturbation([(param, h32)]), T0, device=device)
        _copy_state(a, b, s)
        c = X.Slam(cfg64, X.Perturbation([(param, h64)]), T0, device=device)
        _copy_state(a, c, 1.0)
        a.step(d64[k])
        b.step(d32[k])
        dj = d64[k] * (1.0 + jitter * torch.from_numpy(rng.standard_normal(depths32.shape[1:])).to(device))
        c.step(dj.contiguous())
        done = k + 1
        PA, PB, PC = a.get(X.F_POSE), b.get(X.F_POSE), c.get(X.F_POSE)
        out.append(dict(frame=k, pose_rel_err=_rel(PB[0], PA[0]), grad_rel_err=_rel(PB[1] / h32, PA[1] / h64),
                        pose_spread=_rel(PC[0], PA[0]), grad_spread=_rel(PC[1], PA[1])))
        b.close()
        c.close()
    a.close()
    return out
