"""FP64 CPU reference of the warm-start network (TEST INFRASTRUCTURE ONLY).

The 3-D U-Net of the learned warm start written out with plain PyTorch CPU
operations in float64: 4 levels of 32, 64, 128, 256 channels, two 3x3x3
convolutions (zero padding) + ReLU per level, 2x2x2 average pooling down,
nearest 2x upsampling and channel concatenation [upsampled | skip] up, a
1x1x1 head to one logit per cell, and the mean binary cross-entropy against
the labels (target 1 for solute, phi = -1; solute cells weighted by
pos_weight).  Gradients come from torch's autograd on this float64 graph.

Layouts match the GPU layers' interface: inputs (b, z, y, x, c), weights
(27, cout, cin) with tap = 9 (dz+1) + 3 (dy+1) + (dx+1), logits in (b, z,
y, x) order.  Only tests import this module.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

LEVELS = (32, 64, 128, 256)
IN_C = 32
SPECS = [("e1a", IN_C, 32), ("e1b", 32, 32), ("e2a", 32, 64), ("e2b", 64, 64),
         ("e3a", 64, 128), ("e3b", 128, 128), ("e4a", 128, 256), ("e4b", 256, 256),
         ("d3a", 384, 128), ("d3b", 128, 128), ("d2a", 192, 64), ("d2b", 64, 64),
         ("d1a", 96, 32), ("d1b", 32, 32)]


def to_torch_weight(w):
    """(27, cout, cin) -> (cout, cin, 3, 3, 3) with [kz][ky][kx] = tap 9kz+3ky+kx."""
    w = torch.as_tensor(np.asarray(w, np.float64))
    return w.reshape(3, 3, 3, w.shape[1], w.shape[2]).permute(3, 4, 0, 1, 2).contiguous()


def from_torch_weight(wt):
    return wt.permute(2, 3, 4, 0, 1).reshape(27, wt.shape[0], wt.shape[1]).numpy()


def conv(x, w, b, relu=True):
    """x (b, c, z, y, x) float64; cross-correlation with zero padding 1."""
    y = F.conv3d(x, w, b, padding=1)
    return F.relu(y) if relu else y


def forward(weights, x_cl, labels=None, pos_weight=1.0, grads=False):
    """weights: {name: (w, b)} as numpy (27, cout, cin) / (cout,), "head": ((32,), (1,)).
    x_cl: (b, n, n, n, 32).  Returns dict(logits, loss, grads, dx) as numpy."""
    params = {}
    for name, _, _ in SPECS:
        w, b = weights[name]
        params[name] = (to_torch_weight(w).requires_grad_(grads),
                        torch.as_tensor(np.asarray(b, np.float64)).requires_grad_(grads))
    hw, hb = weights["head"]
    head = (torch.as_tensor(np.asarray(hw, np.float64)).requires_grad_(grads),
            torch.as_tensor(np.asarray(hb, np.float64)).requires_grad_(grads))
    x = torch.as_tensor(np.asarray(x_cl, np.float64)).permute(0, 4, 1, 2, 3).contiguous()

    def c(name, t):
        return conv(t, *params[name])

    s1 = c("e1b", c("e1a", x))
    s2 = c("e2b", c("e2a", F.avg_pool3d(s1, 2)))
    s3 = c("e3b", c("e3a", F.avg_pool3d(s2, 2)))
    b4 = c("e4b", c("e4a", F.avg_pool3d(s3, 2)))
    up = lambda t: F.interpolate(t, scale_factor=2, mode="nearest")  # noqa: E731
    b5 = c("d3b", c("d3a", torch.cat([up(b4), s3], dim=1)))
    b6 = c("d2b", c("d2a", torch.cat([up(b5), s2], dim=1)))
    b7 = c("d1b", c("d1a", torch.cat([up(b6), s1], dim=1)))
    logits = torch.einsum("bczyx,c->bzyx", b7, head[0]) + head[1]
    logits = logits.reshape(-1)
    out = {"logits": logits.detach().numpy()}
    if labels is not None:
        t = torch.as_tensor(np.asarray(labels).reshape(-1) < 0, dtype=torch.float64)
        wt = torch.where(t > 0, torch.full_like(t, float(pos_weight)), torch.ones_like(t))
        loss = F.binary_cross_entropy_with_logits(logits, t, weight=wt, reduction="mean")
        out["loss"] = float(loss.detach())
        if grads:
            loss.backward()
            g = {}
            for name, _, _ in SPECS:
                w, b = params[name]
                g[name] = (from_torch_weight(w.grad), b.grad.numpy())
            g["head"] = (head[0].grad.numpy(), head[1].grad.numpy())
            out["grads"] = g
    return out
