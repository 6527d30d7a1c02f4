"""Helpers shared by the GPU parity tests (HIP path through the C ABI vs the CPU oracle)."""
import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def relerr(x, ref):
    """||x - ref||_inf / max(||ref||_inf, 1e-30); an exact-zero reference requires exact zero."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.abs(ref).max() if ref.size else 0.0
    num = np.abs(x - ref).max() if ref.size else 0.0
    if den == 0.0:
        return 0.0 if num == 0.0 else np.inf
    return num / den


def gpu_pose_to_oracle(P):
    """(..., nc, 4, 4) -> (..., 4, 4, nc)."""
    return np.moveaxis(P, -3, -1)


def gpu_map_to_oracle(M, H, W):
    """(3, nc, H*W) -> (H, W, 3, nc)."""
    nc = M.shape[1]
    return M.reshape(3, nc, H, W).transpose(2, 3, 0, 1)


def oracle_map_to_gpu(M):
    """(H, W, 3, nc) -> (3, nc, H*W)."""
    H, W, _, nc = M.shape
    return M.transpose(2, 3, 0, 1).reshape(3, nc, H * W)


def torch_dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to("cuda:0")


class created_stream:
    """Run the block on a freshly created stream (contexts created inside
    replay their captured frame graph; torch's default stream cannot be
    captured)."""

    def __enter__(self):
        import torch
        self.s = torch.cuda.Stream()
        self.ctx = torch.cuda.stream(self.s)
        self.ctx.__enter__()
        return self.s

    def __exit__(self, *exc):
        self.s.synchronize()
        return self.ctx.__exit__(*exc)
