"""Throughput of the initialiser network's kernels (training steps and
inference) on seeded random inputs, with the MFMA work they carry.

FLOPs per sample: the four convolutions are implicit GEMMs of
(positions x Co) x (Ci*9) each; a forward pass is 2 * sum(Co * Ci * 9 *
positions) plus the small fully connected head, and a training step adds the
input-gradient and weight-gradient GEMMs (about twice the forward).  The
dense bf16 MFMA peak of an MI355X is 2.5 PFLOP/s.

    python -m paper_2405_02187_amd.cnn_bench [--batch 256] [--steps 50]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import xslam as X

CH = (5, 16, 32, 64, 128)
HW = ((60, 80), (30, 40), (15, 20), (8, 10), (4, 5))
PEAK_BF16 = 2.5e15


def conv_flops_per_sample() -> tuple:
    """(forward conv FLOPs, training-step conv FLOPs) per sample."""
    fwd = 0
    for l in range(4):
        pos = HW[l + 1][0] * HW[l + 1][1]
        fwd += 2 * CH[l + 1] * CH[l] * 9 * pos
    # backward: weight gradients of all four layers, input gradients of layers 1..3
    bwd = fwd + sum(2 * CH[l + 1] * CH[l] * 9 * HW[l + 1][0] * HW[l + 1][1] for l in range(1, 4))
    return fwd, fwd + bwd


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--steps", type=int, default=50)
    args = ap.parse_args(argv)
    import torch
    cnn = X.Cnn(max_batch=args.batch)
    rng = np.random.default_rng(0)
    cnn.set_weights((0.05 * rng.standard_normal(cnn.n_params)).astype(np.float32))
    g = torch.Generator(device="cpu").manual_seed(1)
    x = (torch.rand((args.batch, 5, 60, 80), generator=g) * 3.0).to("cuda:0")
    y = (torch.randn((args.batch, 6), generator=g) * 0.01).to("cuda:0")
    for _ in range(3):
        cnn.train_step(x, y, lr=1e-4, want_loss=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cnn.train_step(x, y, lr=1e-4, want_loss=False)
    torch.cuda.synchronize()
    t_train = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cnn.forward(x)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / args.steps
    f_fwd, f_train = conv_flops_per_sample()
    out = dict(batch=args.batch, train_step_ms=1e3 * t_train, forward_ms=1e3 * t_fwd,
               train_samples_per_s=args.batch / t_train, forward_samples_per_s=args.batch / t_fwd,
               conv_tflops_train=f_train * args.batch / t_train / 1e12,
               conv_tflops_forward=f_fwd * args.batch / t_fwd / 1e12,
               frac_of_bf16_peak_train=f_train * args.batch / t_train / PEAK_BF16,
               frac_of_bf16_peak_forward=f_fwd * args.batch / t_fwd / PEAK_BF16)
    print(json.dumps(out), flush=True)
    cnn.close()


if __name__ == "__main__":
    main()
