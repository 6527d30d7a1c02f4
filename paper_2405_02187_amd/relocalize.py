"""Camera relocalisation by the TSDF objective (Sec. 5.2).

Given reference depth images with known camera poses, a query depth image and
an initial estimate of its pose (from any other method):

1. the reference volume M_r is fused from the reference frames near the
   initial estimate, each at its own pose (``xslam_integrate``);
2. the query depth is measured (``xslam_measure``);
3. E(T_q) = sum over voxels of (F_r - F_q)^2, F_q the reference volume with
   the query fused in at T_q, comes with its gradient and Hessian in the
   pose increment from one pass of ``xslam_reloc_energy`` (six hyper-dual
   directions and their 21 pairs: the paper's 6 complex-step and 21
   bicomplex runs of the surface update);
4. the pose is optimised from the estimate: Newton's direction -H^-1 g, the
   gradient direction -g while E exceeds a threshold eta (Newton's method
   depends on its start); or gradient descent alone on the complex-step
   gradient, or on a finite-difference gradient (the paper's comparison).

The threshold is set per contributing voxel: eta = eta_voxel x the number of
voxels that contribute at the initial estimate (E itself scales with the
surface area the query sees).

The paper evaluates on 7-Scenes and its own large-scale captures, with
initial estimates from published relocalisers; neither is available here.
Seeded synthetic sequences (scenegen) stand in: reference frames around the
query on the same trajectory, and an initial estimate that is the true pose
moved by a random rigid transform of fixed size.

    python -m paper_2405_02187_amd.relocalize [--preset c1] [--queries 10]
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import icp_methods as IM
from . import xslam as X

METHODS = ("gd", "gd_fd", "newton")


def build_reference(slam, depths_dev, poses) -> None:
    """Fuse the reference frames (device depth images) at their poses into the
    context's volume (which should start empty)."""
    for d, T in zip(depths_dev, poses):
        slam.integrate(d, pose=np.asarray(T, np.float64))


def objective(slam):
    """E, g, H, count of the relocalisation objective at a pose."""
    return lambda T: slam.reloc_energy(T)


def relocalize(slam, T_init, T_true, method: str = "newton", iters: int = 20, eta_voxel=None,
               radius: float = 0.05, fd_step: float = 1e-3) -> dict:
    """Optimise the query pose (the query already measured, the reference
    volume in place) -> dict(trace, evaluations, T)."""
    f0 = objective(slam)
    n_eval = [0]

    def f(T):
        n_eval[0] += 1
        return f0(T)

    eta = None
    if eta_voxel is not None:
        cnt0 = f(T_init)[3]
        eta = float(eta_voxel) * max(cnt0, 1)
    trace = IM.optimise(f, T_init, T_true, method, iters=iters, radius=radius, eta=eta, fd_step=fd_step)
    return dict(trace=trace, evaluations=n_eval[0], eta=eta)


def perturb(T, t_m: float, r_deg: float, rng) -> np.ndarray:
    """T moved by a random rigid transform: rotation r_deg about a random
    axis, translation t_m along a random direction (left-multiplied)."""
    ax = rng.normal(size=3)
    ax /= np.linalg.norm(ax)
    tr = rng.normal(size=3)
    tr /= np.linalg.norm(tr)
    return IM.se3_exp(np.concatenate([np.radians(r_deg) * ax, t_m * tr])) @ T


def study(preset: dict, depths: np.ndarray, poses_gt: np.ndarray, queries, ref_offsets=(-6, -3, 3, 6),
          t_m: float = 0.03, r_deg: float = 3.0, iters: int = 20, eta_voxel=3e-5, methods=METHODS,
          prec=X.C64, seed: int = 0, radius: float = 0.05, device="cuda:0") -> list:
    """For each query index: a fresh reference volume from the frames at the
    given offsets (at their true poses), the query at its true pose moved by
    (t_m, r_deg), and each method's optimisation.  -> list of dict(query,
    method, t0_m, r0_deg, t_m, r_deg, iterations, evaluations)."""
    import torch
    rng = np.random.default_rng(seed)
    dt = np.float32 if prec == X.C64 else np.float64
    out = []
    for q in queries:
        refs = [q + o for o in ref_offsets if 0 <= q + o < len(depths)]
        T_true = poses_gt[q]
        T_init = perturb(T_true, t_m, r_deg, rng)
        cfg = X.config_from_preset(preset, prec=prec, max_frames=4)
        slam = X.Slam(cfg, X.Perturbation([]), poses_gt[refs[0]], device=device)
        dev = torch.from_numpy(np.ascontiguousarray(depths[refs], dtype=dt)).to(device)
        build_reference(slam, dev, poses_gt[refs])
        slam.measure(torch.from_numpy(np.ascontiguousarray(depths[q], dtype=dt)).to(device))
        for m in methods:
            r = relocalize(slam, T_init, T_true, m, iters=iters, eta_voxel=eta_voxel if m == "newton" else None,
                           radius=radius)
            tr = r["trace"]
            out.append(dict(query=int(q), method=m, t0_m=tr[0]["t_err_m"], r0_deg=tr[0]["r_err_deg"],
                            t_m=tr[-1]["t_err_m"], r_deg=tr[-1]["r_err_deg"], iterations=len(tr) - 1,
                            evaluations=r["evaluations"], E0=tr[0]["E"], E=tr[-1]["E"], count0=tr[0]["count"],
                            count=tr[-1]["count"], newton_steps=sum(1 for x in tr if x.get("step") == "newton"),
                            t_trace=[round(x["t_err_m"], 5) for x in tr],
                            e_voxel_trace=[float("%.4g" % (x["E"] / max(x["count"], 1))) for x in tr]))
        slam.close()
    return out


def summarise(rows: list) -> dict:
    """Median translation / rotation error and recall at (5 cm, 5 deg) per
    method (Table 6's statistics)."""
    s = {}
    for m in sorted({r["method"] for r in rows}):
        rs = [r for r in rows if r["method"] == m]
        s[m] = dict(median_t_cm=100 * float(np.median([r["t_m"] for r in rs])),
                    median_r_deg=float(np.median([r["r_deg"] for r in rs])),
                    recall_5cm_5deg=float(np.mean([(r["t_m"] < 0.05) and (r["r_deg"] < 5.0) for r in rs])),
                    median_iterations=float(np.median([r["iterations"] for r in rs])),
                    median_evaluations=float(np.median([r["evaluations"] for r in rs])))
    rs = [r for r in rows if r["method"] == rows[0]["method"]]
    s["initial"] = dict(median_t_cm=100 * float(np.median([r["t0_m"] for r in rs])),
                        median_r_deg=float(np.median([r["r0_deg"] for r in rs])))
    return s


def main(argv=None):
    import os

    import scenegen as sg
    ap = argparse.ArgumentParser()
    ap.add_argument("--preset", default="c1")
    ap.add_argument("--queries", type=int, default=10)
    ap.add_argument("--t", type=float, default=0.03, help="initial translation error (m)")
    ap.add_argument("--r", type=float, default=3.0, help="initial rotation error (deg)")
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--eta-voxel", type=float, default=3e-5, help="negative: Newton from the start")
    ap.add_argument("--radius", type=float, default=0.05, help="trust radius of a step (rad + m)")
    ap.add_argument("--methods", default=",".join(METHODS))
    ap.add_argument("--prec", default="c64", choices=("c64", "c128"))
    args = ap.parse_args(argv)
    p = sg.preset(args.preset)
    n = 12 * args.queries + 8
    seq = sg.make_sequence(p, n_frames=n)
    depths = seq.depths(workers=min(16, os.cpu_count() or 1))
    qs = [8 + 12 * k for k in range(args.queries)]
    rows = study(p, depths, seq.poses_gt, qs, t_m=args.t, r_deg=args.r, iters=args.iters,
                 eta_voxel=None if args.eta_voxel < 0 else args.eta_voxel, methods=tuple(args.methods.split(",")),
                 prec=X.C64 if args.prec == "c64" else X.C128, radius=args.radius)
    for r in rows:
        print(json.dumps(r), flush=True)
    print(json.dumps(dict(summary=summarise(rows))), flush=True)


if __name__ == "__main__":
    main()
