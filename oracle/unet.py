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


# ----------------------------------------------------- BF16-storage mode

def bf16(t):
    """t rounded to BF16 (8-bit significand, round to nearest, ties to even),
    through FP32 as the GPU layers round their FP32 results; kept as float64."""
    return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def _r(rounding):
    return bf16 if rounding else (lambda t: t)


# The layers of the BF16-storage mode, each on float64 tensors in (b, c, z,
# y, x) order, rounding what the GPU layer stores (rounding=True).

def conv_layer(x, w, b, rounding=True):
    """Stored output of a convolution + bias + ReLU (w: (cout, cin, 3, 3, 3))."""
    return _r(rounding)(F.relu(F.conv3d(x, w, b, padding=1)))


def pool_layer(t, rounding=True):
    """Stored 2x2x2 average."""
    return _r(rounding)(F.avg_pool3d(t, 2))


def upsample(t):
    return F.interpolate(t, scale_factor=2, mode="nearest")


def conv_adjoint(xin, y, dy, w, need_dx=True, rounding=True):
    """Through y = relu(conv(xin) + b): the ReLU adjoint g = dy where y > 0,
    the weight gradient (cout, cin, 3, 3, 3), the bias gradient and the
    stored data gradient at xin (None unless need_dx)."""
    g = torch.where(y > 0, dy, torch.zeros_like(dy))
    gw = torch.nn.grad.conv3d_weight(xin, w.shape, g, padding=1)
    dx = _r(rounding)(torch.nn.grad.conv3d_input(xin.shape, w, g, padding=1)) if need_dx else None
    return dx, gw, g.sum(dim=(0, 2, 3, 4))


def upsample_adjoint(d, rounding=True):
    """Stored sum of the eight children of each half-size cell."""
    return _r(rounding)(F.avg_pool3d(d, 2) * 8.0)


def pool_adjoint_add(dp, dskip, rounding=True):
    """Stored dskip + each cell's share (1/8, stored) of its parent's dp."""
    r = _r(rounding)
    return r(dskip + r(upsample(dp) * 0.125))


def head_layer(b7, hw, hb):
    """Logits (b, z, y, x) of the 1x1x1 head (unrounded, FP32 on the GPU)."""
    return torch.einsum("bczyx,c->bzyx", b7, hw) + hb


def head_adjoint(dlogit, b7, hw, rounding=True):
    """Stored input gradient dlogit w, and the head's weight and bias gradients."""
    dx = _r(rounding)(dlogit.unsqueeze(1) * hw.reshape(1, -1, 1, 1, 1))
    return dx, (dlogit.unsqueeze(1) * b7).sum(dim=(0, 2, 3, 4)), dlogit.sum().reshape(1)


def forward_backward_bf16(weights, x_cl, labels, pos_weight=1.0, rounding=True):
    """The network and its gradients with every tensor the GPU layers store
    in BF16 rounded to BF16 where they store it (rounding=True): the BF16
    weight copies, each convolution's output after bias and ReLU, each pooled
    tensor; in the backward pass the head's input gradient, each data
    gradient, the upsampling adjoint (sum of the eight children) and the
    pooling adjoint (a child's share, then added to the skip gradient).
    Logits, loss, the gradient at the logits, weight and bias gradients stay
    unrounded (the GPU keeps them in FP32).  The backward pass is the chain
    rule written out layer by layer in the GPU's order (no autograd); with
    rounding=False it is the exact gradient of forward().  Arithmetic in
    float64.  Returns dict(logits, loss, grads) as numpy."""
    r = _r(rounding)
    W = {}
    for name, _, _ in SPECS:
        w, b = weights[name]
        W[name] = (r(to_torch_weight(w)), torch.as_tensor(np.asarray(b, np.float64)))
    hw = torch.as_tensor(np.asarray(weights["head"][0], np.float64))
    hb = torch.as_tensor(np.asarray(weights["head"][1], np.float64))
    x = torch.as_tensor(np.asarray(x_cl, np.float64)).permute(0, 4, 1, 2, 3).contiguous()

    def cf(name, t):
        return conv_layer(t, *W[name], rounding=rounding)

    a = {"x": x}
    a["a1"] = cf("e1a", x)
    a["s1"] = cf("e1b", a["a1"])
    a["p1"] = pool_layer(a["s1"], rounding)
    a["a2"] = cf("e2a", a["p1"])
    a["s2"] = cf("e2b", a["a2"])
    a["p2"] = pool_layer(a["s2"], rounding)
    a["a3"] = cf("e3a", a["p2"])
    a["s3"] = cf("e3b", a["a3"])
    a["p3"] = pool_layer(a["s3"], rounding)
    a["a4"] = cf("e4a", a["p3"])
    a["b4"] = cf("e4b", a["a4"])
    a["c3"] = torch.cat([upsample(a["b4"]), a["s3"]], dim=1)
    a["a5"] = cf("d3a", a["c3"])
    a["b5"] = cf("d3b", a["a5"])
    a["c2"] = torch.cat([upsample(a["b5"]), a["s2"]], dim=1)
    a["a6"] = cf("d2a", a["c2"])
    a["b6"] = cf("d2b", a["a6"])
    a["c1"] = torch.cat([upsample(a["b6"]), a["s1"]], dim=1)
    a["a7"] = cf("d1a", a["c1"])
    a["b7"] = cf("d1b", a["a7"])
    logits = head_layer(a["b7"], hw, hb)
    lf = logits.reshape(-1)
    t = torch.as_tensor(np.asarray(labels).reshape(-1) < 0, dtype=torch.float64)
    wt = torch.where(t > 0, torch.full_like(t, float(pos_weight)), torch.ones_like(t))
    P = lf.numel()
    # mean weighted BCE and its gradient at the logits
    loss = (wt * (F.softplus(-lf.abs()) + lf.clamp(min=0) - lf * t)).sum() / P
    dlogit = (wt * (torch.sigmoid(lf) - t) / P).reshape(logits.shape)

    db7, hgw, hgb = head_adjoint(dlogit, a["b7"], hw, rounding)
    grads = {"head": (hgw.numpy(), hgb.numpy())}

    def cb(name, xin, y, dy, need_dx=True):
        dx, gw, gb = conv_adjoint(xin, y, dy, W[name][0], need_dx, rounding)
        grads[name] = (from_torch_weight(gw), gb.numpy())
        return dx

    c1, c2, c3, c4 = LEVELS
    da7 = cb("d1b", a["a7"], a["b7"], db7)
    dc1 = cb("d1a", a["c1"], a["a7"], da7)
    db6, ds1 = upsample_adjoint(dc1[:, :c2], rounding), dc1[:, c2:]
    da6 = cb("d2b", a["a6"], a["b6"], db6)
    dc2 = cb("d2a", a["c2"], a["a6"], da6)
    db5, ds2 = upsample_adjoint(dc2[:, :c3], rounding), dc2[:, c3:]
    da5 = cb("d3b", a["a5"], a["b5"], db5)
    dc3 = cb("d3a", a["c3"], a["a5"], da5)
    db4, ds3 = upsample_adjoint(dc3[:, :c4], rounding), dc3[:, c4:]
    da4 = cb("e4b", a["a4"], a["b4"], db4)
    dp3 = cb("e4a", a["p3"], a["a4"], da4)
    ds3 = pool_adjoint_add(dp3, ds3, rounding)
    da3 = cb("e3b", a["a3"], a["s3"], ds3)
    dp2 = cb("e3a", a["p2"], a["a3"], da3)
    ds2 = pool_adjoint_add(dp2, ds2, rounding)
    da2 = cb("e2b", a["a2"], a["s2"], ds2)
    dp1 = cb("e2a", a["p1"], a["a2"], da2)
    ds1 = pool_adjoint_add(dp1, ds1, rounding)
    da1 = cb("e1b", a["a1"], a["s1"], ds1)
    cb("e1a", a["x"], a["a1"], da1, need_dx=False)
    return {"logits": lf.numpy(), "loss": float(loss), "grads": grads}
