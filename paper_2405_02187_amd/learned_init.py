"""Training data, training and evaluation of the learned ICP initialiser.

Pairs come from the frame step itself: running a sequence (FP32, no
derivatives), after every frame k the library returns the network-input parts
of that frame (its depth at level 3 and the raycast model maps in its camera
frame).  A pair (k - s, k) is the depth of frame k with the model maps of
frame k - s; its label is the converged relative pose log(T_{k-s}^-1 T_k)
(right increment in camera k - s).  Training and inference run in the
library's kernels; this module only arranges data.
"""
from __future__ import annotations

import numpy as np

from . import xslam as X


def se3_log(T: np.ndarray) -> np.ndarray:
    """(phi, rho) with T = exp([phi, rho]) (the inverse of the pose exponential)."""
    from scipy.spatial.transform import Rotation
    R, t = T[:3, :3], T[:3, 3]
    phi = Rotation.from_matrix(R).as_rotvec()
    th2 = float(phi @ phi)
    if th2 < 1e-8:
        B, Cc = 0.5 - th2 / 24.0, 1.0 / 6.0 - th2 / 120.0
    else:
        th = np.sqrt(th2)
        B, Cc = (1 - np.cos(th)) / th2, (th - np.sin(th)) / (th2 * th)
    K = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    V = np.eye(3) + B * K + Cc * K @ K
    return np.concatenate([phi, np.linalg.solve(V, t)])


def run_sequence_parts(cfg, depths_dev, T0, frame_step: int = 1):
    """Run frames 0, s, 2s, ...; -> (poses (n,4,4), depth parts (n,1,60,80), model parts (n,4,60,80))."""
    import torch
    slam = X.Slam(cfg, X.Perturbation([]), T0)
    dparts, mparts = [], []
    idx = list(range(0, depths_dev.shape[0], frame_step))
    for k in idx:
        slam.step(depths_dev[k])
        d, m = slam.cnn_parts()
        dparts.append(d)
        mparts.append(m)
    poses = slam.get(X.F_POSES)[:, 0]
    cnt = slam.get(X.F_COUNTERS)
    slam.close()
    return poses, torch.stack(dparts), torch.stack(mparts), cnt


def make_pairs(poses, dparts, mparts, max_step: int = 8):
    """All pairs (k - s, k), 1 <= s <= max_step -> inputs (P,5,60,80), labels (P,6) (torch, device)."""
    import torch
    xs, ys = [], []
    n = len(poses)
    for s in range(1, max_step + 1):
        for k in range(s, n):
            xs.append(torch.cat([dparts[k], mparts[k - s]], 0))
            rel = np.linalg.inv(poses[k - s]) @ poses[k]
            ys.append(se3_log(rel))
    X_ = torch.stack(xs)
    Y_ = torch.tensor(np.array(ys), dtype=torch.float32, device=X_.device)
    return X_, Y_


def train(net: "X.Cnn", Xd, Yd, steps: int, batch: int = 256, lr: float = 1e-3, seed: int = 0):
    """Adam on random minibatches of the pairs; -> list of losses."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    losses = []
    n = Xd.shape[0]
    for _ in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), generator=g).to(Xd.device)
        xb = Xd.index_select(0, idx).contiguous()
        yb = Yd.index_select(0, idx).contiguous()
        losses.append(net.train_step(xb, yb, lr=lr))
    return losses


def evaluate(cfg_base, depths_dev, T0, gt, frame_step: int, net=None):
    """Track every frame_step-th frame with constant velocity (net None) or the
    network initialiser; -> dict(first converged pass per frame, trajectory
    error, network use rate)."""
    import ctypes as C
    cfg = X.xslam_config.from_buffer_copy(cfg_base)
    cfg.icp.init = 2 if net is not None else 1
    slam = X.Slam(cfg, X.Perturbation([]), T0)
    if net is not None:
        slam.set_cnn(net)
    idx = list(range(0, depths_dev.shape[0], frame_step))
    for k in idx:
        slam.step(depths_dev[k])
    cnt = slam.get(X.F_COUNTERS)[1:]
    poses = slam.get(X.F_POSES)[:, 0]
    err = np.sqrt(np.mean(np.sum((poses[:, :3, 3] - gt[idx][:, :3, 3]) ** 2, axis=1)))
    conv = cnt[:, 32].astype(float)
    conv[conv == 0] = float(sum(cfg.icp.iters)) + 1          # never converged
    out = dict(conv_pass_mean=float(conv.mean()), traj_err=float(err), net_used=float(cnt[:, 33].mean()),
               lost=int(cnt[:, 0].sum()))
    slam.close()
    return out
