"""Launch-shape autotuner with a JSON cache.

The library times the stages it can re-run without changing state (raycast
tile, ICP grid per level; ``Slam.autotune``).  The fusion grid changes the
TSDF when it runs, so it is tuned here on real frames: consecutive steps of
the sequence with different grids, timed by the library's per-kernel event
timer (no result depends on the fusion grid).  Chosen shapes are cached per
workload shape (image size, volume, precision, directions, Hessian size).
"""
from __future__ import annotations

import json
import os

from . import xslam as X

FUSE_GRIDS = (4096, 2048, 1024, 512)


def key(slam: "X.Slam") -> str:
    c = slam.cfg
    prec = "c128" if c.prec == X.C128 else "c64"
    dims = "x".join(str(int(d)) for d in c.vol.dim)
    return f"{c.cam.width}x{c.cam.height}_{dims}_{prec}_D{slam.D}_Q{slam.Q}"


def load(path: str) -> dict:
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save(path: str, cache: dict) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(slam: "X.Slam", shapes: dict) -> None:
    slam.set_launch(ray_tile=tuple(shapes["ray_tile"]), icp_blocks=tuple(shapes["icp_blocks"]),
                    fuse_blocks=int(shapes["fuse_blocks"]))


def tune(slam: "X.Slam", frames, reps: int = 20, fuse_frames_per_grid: int = 2) -> dict:
    """Tune on a context that has stepped at least one frame.  ``frames`` is an
    iterable of device depth frames that continue the sequence (used for the
    fusion grid: len(FUSE_GRIDS) * fuse_frames_per_grid of them are stepped).
    -> dict(ray_tile, icp_blocks, fuse_blocks, ms)."""
    shapes, ms = slam.autotune(reps)
    it = iter(frames)
    t_fuse = {g: 0.0 for g in FUSE_GRIDS}
    slam.set_timing(True)
    for _ in range(fuse_frames_per_grid):
        for g in FUSE_GRIDS:
            slam.set_launch(fuse_blocks=g)
            before = slam.kernel_times()[0][2]
            slam.step(next(it))
            t_fuse[g] += slam.kernel_times()[0][2] - before
    slam.set_timing(False)
    best_fuse = min(FUSE_GRIDS, key=lambda g: t_fuse[g])
    slam.set_launch(fuse_blocks=best_fuse)
    out = slam.get_launch()
    out["ms"] = dict(raycast=float(ms[0]), icp=[float(x) for x in ms[1:]],
                     fuse={str(g): t_fuse[g] / fuse_frames_per_grid for g in FUSE_GRIDS})
    out["ray_tile"] = list(out["ray_tile"])
    out["icp_blocks"] = list(out["icp_blocks"])
    return out


def tuned(slam: "X.Slam", frames, cache_path: str | None = None, reps: int = 20) -> dict:
    """Cached shapes for this workload if present (applied), else tune, store
    and return them."""
    cache = load(cache_path) if cache_path else {}
    k = key(slam)
    if k in cache:
        apply(slam, cache[k])
        return cache[k]
    out = tune(slam, frames, reps=reps)
    if cache_path:
        cache[k] = out
        save(cache_path, cache)
    return out


def frames_needed(fuse_frames_per_grid: int = 2) -> int:
    return len(FUSE_GRIDS) * fuse_frames_per_grid


__all__ = ["key", "load", "save", "apply", "tune", "tuned", "frames_needed", "FUSE_GRIDS"]
