"""Several independent CSFD sequences of uneven size advanced together.

Each instance is its own context (volume, image size, directions).  Two ways
to step them, one frame of every unfinished instance per round:

* streams: each context on its own HIP stream, its frame step launched by
  itself, so the latency-bound ICP passes and small volumes of one instance
  overlap with the work of the others;
* grouped: contexts of one shape (number of directions) on one stream are
  stepped by grouped launches, one grid per stage for all of them, each
  context bringing its descriptor and its own grid of work items; a shape's
  contexts are dealt to groups of at most group_size, each group on its own
  stream, and the groups overlap.

Throughput is the aggregate frames x directions over the wall time of the
whole batch; latency is the device time of each frame step under that load
(HIP events on its stream; grouped: the group's step).
"""
from __future__ import annotations

import time

import numpy as np

from . import xslam as X


def make_instances(presets, workers: int = 16, frame_cap: int | None = None, device="cuda:0"):
    """Render every instance's depth (and noise tangent when it perturbs the
    depth) and move it to the device.  -> list of dicts."""
    import torch
    import scenegen as sg
    out = []
    for p in presets:
        n = p["n_frames"] if frame_cap is None else min(p["n_frames"], frame_cap)
        seq = sg.make_sequence(p, n_frames=n)
        if X.P_DEPTH in p["dirs"]:
            d, t = seq.depths_and_tangents(n, workers=workers)
            tan = torch.from_numpy(t.astype(np.float32)).to(device)
        else:
            d, tan = seq.depths(n, workers=workers), None
        out.append(dict(preset=p, n=n, T0=seq.poses_gt[0], gt=seq.poses_gt,
                        depth=torch.from_numpy(d.astype(np.float32)).to(device), tangent=tan))
    return out


def make_context(inst, stream=None):
    import torch
    p = inst["preset"]
    cfg = X.config_from_preset(p, prec=X.C64, max_frames=inst["n"])
    pert = X.Perturbation([(q, p["h"]) for q in p["dirs"]])
    if stream is None:
        return X.Slam(cfg, pert, inst["T0"])
    with torch.cuda.stream(stream):
        return X.Slam(cfg, pert, inst["T0"])


def shape_of(inst):
    return len(inst["preset"]["dirs"])


def group_streams(instances, group_size: int):
    """Stream index of every instance in grouped mode: each shape's instances
    (in order) dealt round-robin to ceil(count / group_size) groups."""
    out, nxt = [None] * len(instances), 0
    for q in sorted({shape_of(inst) for inst in instances}):
        idx = [i for i, inst in enumerate(instances) if shape_of(inst) == q]
        ng = -(-len(idx) // group_size)
        for k, i in enumerate(idx):
            out[i] = nxt + k % ng
        nxt += ng
    return out


def run_batch(instances, n_streams: int | None = None, grouped: bool = False, persist: int = 0,
              group_size: int = 32):
    """All instances to the end of their sequences, together.  -> dict with
    aggregate frames*directions/s, per-frame latency percentiles and the
    contexts (caller closes them).  grouped: grouped launches, groups of at
    most group_size instances of one shape, one stream per group (n_streams
    is ignored)."""
    import torch
    n = len(instances)
    if grouped:
        gs = group_streams(instances, group_size)
        streams = [torch.cuda.Stream() for _ in range(max(gs) + 1)]
        slams = [make_context(inst, streams[g]) for inst, g in zip(instances, gs)]
        n_streams = len(streams)
    else:
        n_streams = n if n_streams is None else n_streams
        streams = [torch.cuda.Stream() for _ in range(n_streams)]
        slams = [make_context(inst, streams[i % n_streams]) for i, inst in enumerate(instances)]
    batch = X.Batch(slams, grouped=grouped, persist=persist)
    lat = []
    n_max = max(inst["n"] for inst in instances)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n_max):
        active = [k < inst["n"] for inst in instances]
        depths = [inst["depth"][k] if a else None for inst, a in zip(instances, active)]
        tans = [inst["tangent"][k] if (a and inst["tangent"] is not None) else None
                for inst, a in zip(instances, active)]
        batch.step(depths, tans, active)
        if k % 8 == 7 or k == n_max - 1:
            ms = batch.latency()               # waits for this round (keeps the queues short)
            lat.extend(float(x) for x in ms if x >= 0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    work = sum(inst["n"] * len(inst["preset"]["dirs"]) for inst in instances)
    frames = sum(inst["n"] for inst in instances)
    batch.close()
    lat = np.array(lat)
    return dict(value=work / wall, frames=frames, frames_x_dirs=work, wall_s=wall, streams=n_streams,
                mode="grouped" if grouped else "streams", persist=persist,
                group_size=group_size if grouped else None,
                latency_ms=dict(p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99)),
                                sampled_rounds=int(len(lat))),
                slams=slams)


def run_alone(instance):
    """One instance by itself on the current stream -> (slam, wall seconds)."""
    import torch
    slam = make_context(instance)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(instance["n"]):
        slam.step(instance["depth"][k], None if instance["tangent"] is None else instance["tangent"][k])
    torch.cuda.synchronize()
    return slam, time.perf_counter() - t0
