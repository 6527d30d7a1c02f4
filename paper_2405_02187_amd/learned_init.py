"""Training data, training and evaluation of the learned ICP initialiser.

Pairs come from the frame step itself: running a sequence (FP32, no
derivatives), after every frame k the library returns the network-input parts
of that frame (its depth at pyramid level 3 and the raycast model maps in its
camera frame).  A pair (k - s, k) is the depth of frame k with the model maps
of frame k - s; its label is the converged relative pose log(T_{k-s}^-1 T_k)
(the right increment in camera k - s).  Training and inference run in the
library's kernels; this module only arranges data.

``python -m paper_2405_02187_amd.learned_init`` trains on seeded sequences
and compares, on held-out sequences tracked at several frame steps, the
network initialiser (with its residual test) against constant velocity:
ICP passes to convergence (|update| < 1e-6) and trajectory error.
"""
from __future__ import annotations

import argparse
import json
import time

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
    """Run frames 0, s, 2s, ...; -> (poses (n,4,4), depth parts (n,1,60,80),
    model parts (n,4,60,80), counters)."""
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


class PairSet:
    """Pairs (k - s, k), 1 <= s <= max_step, of one or more sequences, held as
    indices into the per-frame parts (device) with their labels."""

    def __init__(self):
        self.dparts, self.mparts = [], []
        self.cur, self.prev, self.labels = [], [], []
        self.base = 0

    def add(self, poses, dparts, mparts, max_step: int = 8, ok=None):
        n = len(poses)
        ok = np.ones(n, dtype=bool) if ok is None else ok
        for s in range(1, max_step + 1):
            for k in range(s, n):
                if not (ok[k] and ok[k - s]):
                    continue
                self.cur.append(self.base + k)
                self.prev.append(self.base + k - s)
                self.labels.append(se3_log(np.linalg.inv(poses[k - s]) @ poses[k]))
        self.dparts.append(dparts)
        self.mparts.append(mparts)
        self.base += n

    def finalize(self):
        import torch
        self.D = torch.cat(self.dparts)
        self.M = torch.cat(self.mparts)
        dev = self.D.device
        self.icur = torch.tensor(self.cur, dtype=torch.int64, device=dev)
        self.iprev = torch.tensor(self.prev, dtype=torch.int64, device=dev)
        self.Y = torch.tensor(np.array(self.labels), dtype=torch.float32, device=dev)
        return self

    def __len__(self):
        return len(self.cur)

    def batch(self, idx):
        import torch
        x = torch.cat([self.D.index_select(0, self.icur[idx]), self.M.index_select(0, self.iprev[idx])], 1)
        return x.contiguous(), self.Y.index_select(0, idx).contiguous()


def make_pairs(poses, dparts, mparts, max_step: int = 8):
    """All pairs of one sequence -> inputs (P,5,60,80), labels (P,6) (device)."""
    import torch
    ps = PairSet()
    ps.add(poses, dparts, mparts, max_step)
    ps.finalize()
    return ps.batch(torch.arange(len(ps), device=ps.D.device))


def train(net: "X.Cnn", data, Yd=None, steps: int = 1000, batch: int = 256, lr: float = 1e-3, seed: int = 0):
    """Adam on random minibatches.  ``data`` is a PairSet, or inputs with
    labels ``Yd``.  -> list of losses."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    losses = []
    if isinstance(data, PairSet):
        n = len(data)
        get = data.batch
        dev = data.D.device
    else:
        n = data.shape[0]
        dev = data.device

        def get(idx):
            return data.index_select(0, idx).contiguous(), Yd.index_select(0, idx).contiguous()
    for _ in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), generator=g).to(dev)
        xb, yb = get(idx)
        losses.append(net.train_step(xb, yb, lr=lr))
    return losses


def evaluate(cfg_base, depths_dev, T0, gt, frame_step, net=None):
    """Track every frame_step-th frame (or the frames listed in frame_step)
    with constant velocity (net None) or the network initialiser; -> dict(mean
    first converged ICP pass per tracked frame (passes + 1 when none
    converged), trajectory error, network use rate, lost frames)."""
    cfg = X.xslam_config.from_buffer_copy(cfg_base)
    cfg.icp.init = 2 if net is not None else 1
    slam = X.Slam(cfg, X.Perturbation([]), T0)
    if net is not None:
        slam.set_cnn(net)
    if isinstance(frame_step, int):
        idx = list(range(0, depths_dev.shape[0], frame_step))
    else:
        idx = [int(k) for k in frame_step]
    for k in idx:
        slam.step(depths_dev[k])
    cnt = slam.get(X.F_COUNTERS)[1:]
    poses = slam.get(X.F_POSES)[:, 0]
    err = np.sqrt(np.mean(np.sum((poses[:, :3, 3] - gt[idx][:, :3, 3]) ** 2, axis=1)))
    conv = cnt[:, 32].astype(float)
    conv[conv == 0] = float(sum(cfg.icp.iters)) + 1          # never converged
    out = dict(conv_pass_mean=float(conv.mean()), converged_frac=float((cnt[:, 32] > 0).mean()),
               traj_err=float(err), net_used=float(cnt[:, 33].mean()), lost=int(cnt[:, 0].sum()))
    slam.close()
    return out


def _sequence(sg, torch, preset, seed, n, workers=16):
    p = sg.preset(preset, seed=seed)
    s = sg.make_sequence(p, n_frames=n)
    d = torch.from_numpy(s.depths(workers=workers).astype(np.float32)).cuda()
    return p, s, d


def main(argv=None):
    import torch
    import scenegen as sg
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-preset", default="c2", help="scene / volume preset of the training sequences")
    ap.add_argument("--train-seeds", type=int, default=16)
    ap.add_argument("--test-seeds", type=int, default=4)
    ap.add_argument("--frames", type=int, default=300)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--max-step", type=int, default=8)
    ap.add_argument("--frame-steps", default="1,3,6")
    ap.add_argument("--out", default=None, help="JSON report path")
    a = ap.parse_args(argv)
    t0 = time.perf_counter()
    ps = PairSet()
    lost_train = 0
    for i in range(a.train_seeds):
        p, s, d = _sequence(sg, torch, a.train_preset, 1000 + i, a.frames)
        cfg = X.config_from_preset(p, prec=X.C64, max_frames=a.frames)
        poses, dp, mp, cnt = run_sequence_parts(cfg, d, s.poses_gt[0])
        # pairs only between frames that tracked (label quality): not lost and
        # within 5 cm of ground truth
        ok = (cnt[:, 0] == 0) & (np.linalg.norm(poses[:, :3, 3] - s.poses_gt[:, :3, 3], axis=1) < 0.05)
        ps.add(poses, dp, mp, a.max_step, ok)
        lost_train += int(cnt[:, 0].sum())
        print(f"train seed {1000 + i}: {int(ok.sum())}/{a.frames} frames usable, {len(ps)} pairs", flush=True)
        del d
    ps.finalize()
    t_data = time.perf_counter() - t0
    net = X.Cnn(max_batch=a.batch)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(0, spawn_key=(7,))))
    w0 = []
    for shp in net_shapes():
        if len(shp) == 1:
            w0.append(np.zeros(shp))
        else:
            lim = np.sqrt(6.0 / int(np.prod(shp[1:])))
            w0.append(rng.uniform(-lim, lim, size=shp))
    net.set_weights(np.concatenate([w.reshape(-1) for w in w0]))
    t1 = time.perf_counter()
    losses = train(net, ps, steps=a.steps, batch=a.batch, lr=a.lr)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    print(f"trained {a.steps} steps in {t_train:.1f}s: loss {np.mean(losses[:20]):.1f} -> {np.mean(losses[-20:]):.2f}",
          flush=True)
    report = dict(pairs=len(ps), train_preset=a.train_preset, train_seeds=a.train_seeds, frames=a.frames,
                  lost_train_frames=lost_train, steps=a.steps, batch=a.batch,
                  loss_first=float(np.mean(losses[:20])), loss_last=float(np.mean(losses[-20:])),
                  train_s=t_train, data_s=t_data, samples_per_s=a.steps * a.batch / t_train, tests=[])
    for j in range(a.test_seeds):
        p, s, d = _sequence(sg, torch, "c1", 2000 + j, a.frames)
        cfg = X.config_from_preset(p, prec=X.C64, max_frames=a.frames)
        # regular steps, and irregular ones (dropped frames: gaps of 1..6
        # frames, seeded) where a constant velocity extrapolates the wrong gap
        rng = np.random.default_rng(2000 + j)
        irregular = np.cumsum(np.concatenate([[0], rng.integers(1, 7, size=a.frames)]))
        irregular = irregular[irregular < a.frames]
        for fs in [int(x) for x in a.frame_steps.split(",")] + ["irregular"]:
            steps = irregular if fs == "irregular" else fs
            cv = evaluate(cfg, d, s.poses_gt[0], s.poses_gt, steps, None)
            nn = evaluate(cfg, d, s.poses_gt[0], s.poses_gt, steps, net)
            report["tests"].append(dict(seed=2000 + j, frame_step=fs, constant_velocity=cv, network=nn))
            print(f"test seed {2000 + j} step {fs}: cv {cv}  net {nn}", flush=True)
        del d
    net.close()
    # per frame step: means over the held-out seeds
    summary = {}
    for fs in sorted({str(t["frame_step"]) for t in report["tests"]}):
        ts = [t for t in report["tests"] if str(t["frame_step"]) == fs]
        summary[fs] = {k: {m: float(np.mean([t[k][m] for t in ts])) for m in ts[0][k]}
                       for k in ("constant_velocity", "network")}
    report["summary"] = summary
    print("summary over held-out seeds:", json.dumps(summary), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(report, f, indent=1)
    print(json.dumps({k: v for k, v in report.items() if k != "tests"}))
    return report


def net_shapes():
    ch = [5, 16, 32, 64, 128]
    s = []
    for i in range(4):
        s += [(ch[i + 1], ch[i], 3, 3), (ch[i + 1],)]
    return s + [(64, 128), (64,), (6, 64), (6,)]


if __name__ == "__main__":
    main()
