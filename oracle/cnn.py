"""FP64 oracle of the learned ICP initialiser -- TEST INFRASTRUCTURE ONLY.

The network proposes the initial pose increment of ICP from coarse maps: a
5x60x80 input (current depth; raycast depth and raycast normal of the previous
frame in its camera frame; invalid pixels 0), four 3x3 stride-2 padding-1
convolutions with ReLU (5->16->32->64->128 channels), global average pooling,
then 128->64 (ReLU) -> 6, giving the se(3) increment (phi, rho).  The loss of a
batch is the mean over samples of |diag(1/0.01) (xi_hat - xi)|^2.  Training
uses Adam.  This file writes those definitions out with plain numpy loops over
kernel offsets; backward passes are derived by hand.  Only tests and the
benchmark's CPU baseline use it.

``quant=bf16_round`` (forward and backward) rounds to bfloat16 at the points
where a bf16 implementation stores values: the network input, the
convolution weights, every post-ReLU activation, and the gradient with
respect to every convolution output (biases and the fully connected layers
stay in full precision).  Arithmetic stays FP64.  The ReLU
masks are decisions taken by floating point, so a bf16 implementation is
compared with this mode (both take the masks from bf16-stored values); with
``quant=None`` everything is FP64.
"""
from __future__ import annotations

import numpy as np

CH = [5, 16, 32, 64, 128]
FC = [128, 64, 6]
IN_H, IN_W = 60, 80
LOSS_SCALE = 1.0 / 0.01


def out_size(n: int) -> int:
    return (n + 2 - 3) // 2 + 1


def shapes():
    """Parameter shapes in a fixed order: conv weights/biases, then FC."""
    s = []
    for i in range(4):
        s += [(CH[i + 1], CH[i], 3, 3), (CH[i + 1],)]
    s += [(FC[1], FC[0]), (FC[1],), (FC[2], FC[1]), (FC[2],)]
    return s


def n_params() -> int:
    return int(sum(np.prod(x) for x in shapes()))


def init_params(seed: int = 0):
    """He-uniform init from a seeded PCG64 stream (inputs to both sides)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(7,))))
    out = []
    for shp in shapes():
        if len(shp) == 1:
            out.append(np.zeros(shp))
        else:
            fan_in = int(np.prod(shp[1:]))
            lim = np.sqrt(6.0 / fan_in)
            out.append(rng.uniform(-lim, lim, size=shp))
    return out


def bf16_round(a):
    """Round to the nearest bfloat16 (the upper 16 bits of an IEEE binary32,
    ties to even), returned as float64.  The value is first rounded to
    binary32."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    bits = a32.view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def _ident(a):
    return a


def conv_s2(x, w, b):
    """x (N,Ci,H,W), w (Co,Ci,3,3), stride 2, zero padding 1 -> (N,Co,Ho,Wo)."""
    N, Ci, H, W = x.shape
    Ho, Wo = out_size(H), out_size(W)
    xp = np.zeros((N, Ci, H + 2, W + 2))
    xp[:, :, 1:H + 1, 1:W + 1] = x
    y = np.zeros((N, w.shape[0], Ho, Wo)) + b[None, :, None, None]
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, :, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2]          # (N,Ci,Ho,Wo)
            y += np.einsum("nchw,oc->nohw", patch, w[:, :, ky, kx])
    return y


def conv_s2_backward(x, w, dy):
    """Gradients of conv_s2 w.r.t. x, w, b given dy."""
    N, Ci, H, W = x.shape
    Ho, Wo = dy.shape[2], dy.shape[3]
    xp = np.zeros((N, Ci, H + 2, W + 2))
    xp[:, :, 1:H + 1, 1:W + 1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, :, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2]
            dw[:, :, ky, kx] = np.einsum("nohw,nchw->oc", dy, patch)
            dxp[:, :, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2] += np.einsum("nohw,oc->nchw", dy, w[:, :, ky, kx])
    db = dy.sum(axis=(0, 2, 3))
    return dxp[:, :, 1:H + 1, 1:W + 1], dw, db


def forward(params, x, quant=None):
    """-> (xi (N,6), cache)."""
    q = quant or _ident
    h = q(x)
    acts = [h]
    pre = []
    convw = [(q(params[2 * i]), params[2 * i + 1]) for i in range(4)]
    for i in range(4):
        z = conv_s2(h, *convw[i])
        pre.append(z)
        h = q(np.maximum(z, 0.0))
        acts.append(h)
    g = h.mean(axis=(2, 3))                                                  # (N,128)
    z5 = g @ params[8].T + params[9]
    h5 = np.maximum(z5, 0.0)
    xi = h5 @ params[10].T + params[11]
    return xi, dict(acts=acts, pre=pre, g=g, z5=z5, h5=h5, convw=convw, quant=q)


def loss(xi, label):
    d = (xi - label) * LOSS_SCALE
    return float(np.mean(np.sum(d * d, axis=1)))


def backward(params, cache, xi, label):
    """Gradients of loss w.r.t. every parameter (same order as shapes())."""
    N = xi.shape[0]
    dxi = 2.0 * (xi - label) * LOSS_SCALE ** 2 / N
    grads = [None] * 12
    grads[10] = dxi.T @ cache["h5"]
    grads[11] = dxi.sum(0)
    dh5 = dxi @ params[10]
    dz5 = dh5 * (cache["z5"] > 0)
    grads[8] = dz5.T @ cache["g"]
    grads[9] = dz5.sum(0)
    dg = dz5 @ params[8]
    h4 = cache["acts"][4]
    q = cache["quant"]
    dh = np.broadcast_to(dg[:, :, None, None] / (h4.shape[2] * h4.shape[3]), h4.shape).copy()
    for i in range(3, -1, -1):
        dz = q(dh * (cache["pre"][i] > 0))
        dx, dw, db = conv_s2_backward(cache["acts"][i], cache["convw"][i][0], dz)
        grads[2 * i], grads[2 * i + 1] = dw, db
        dh = dx
    return grads


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected, t starting at 1); returns new lists."""
    P, M, V = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = b1 * mm + (1 - b1) * g
        vv = b2 * vv + (1 - b2) * g * g
        mh = mm / (1 - b1 ** t)
        vh = vv / (1 - b2 ** t)
        P.append(p - lr * mh / (np.sqrt(vh) + eps))
        M.append(mm)
        V.append(vv)
    return P, M, V
