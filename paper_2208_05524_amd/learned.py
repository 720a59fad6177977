"""The learned warm start: a 3-D U-Net that predicts the equilibrium labels
of the binary level-set relaxation from the atoms, trained on labels the
relaxation itself produced.  Not part of the paper (which starts from a
loose or tight sphere); the relaxation always finishes from the predicted
labels, so a poor prediction costs sweeps, never correctness of the
relaxation.

Architecture: 4 levels with 32, 64, 128, 256 channels, two 3x3x3
convolutions + ReLU per level, 2x2x2 average pooling down, nearest 2x
upsampling + channel concatenation with the skip up, a 1x1x1 head to one
logit per cell (solute where positive).  Input: 32 channels on the cell
grid, of which channel 0 is the Gaussian-smeared atom density and channel 1
the smeared charge (vesis_nn_featurize), the rest zero; inference takes the
first 16 of them (the same logits, half the first convolution's work).

Every layer runs in the library's HIP kernels (include/vesis_nn.h); torch
tensors serve only as device memory.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import nn as N

IN_C = 32
# Inference reads the input as one 16-channel chunk: only channels 0 and 1
# are ever nonzero, so the first convolution's second chunk of 16 input
# channels adds exact zeros, and leaving it out changes no logit.
INFER_C = 16
LEVELS = (32, 64, 128, 256)


def layer_specs():
    """(name, cin, cout) of every 3x3x3 convolution, in forward order."""
    c1, c2, c3, c4 = LEVELS
    return [("e1a", IN_C, c1), ("e1b", c1, c1), ("e2a", c1, c2), ("e2b", c2, c2),
            ("e3a", c2, c3), ("e3b", c3, c3), ("e4a", c3, c4), ("e4b", c4, c4),
            ("d3a", c4 + c3, c3), ("d3b", c3, c3), ("d2a", c3 + c2, c2), ("d2b", c2, c2),
            ("d1a", c2 + c1, c1), ("d1b", c1, c1)]


def init_weights(seed: int = 0):
    """He-uniform weights from the seeded input generators, zero biases:
    {name: (w (27, cout, cin) float32, b (cout,) float32)}, head included."""
    import synth
    return synth.conv_weights(layer_specs(), LEVELS[0], seed)


class UNet:
    """Parameters, activations and gradients on one device; forward,
    backward and Adam through the library's kernels."""

    def __init__(self, size: int, batch: int = 1, device: int = 0, seed: int = 0,
                 weights=None, train: bool = True):
        """train=False: inference only (no gradients, optimiser state or
        weight-gradient scratch)."""
        import torch
        if size % 8:
            raise ValueError("grid size must be a multiple of 8 (three poolings)")
        self.t = torch
        self.dev = torch.device("cuda", device)
        self.L = N.lib()
        self.n, self.b = size, batch
        w0 = weights if weights is not None else init_weights(seed)
        self.specs = layer_specs()
        self.p = {}
        f32 = dict(dtype=torch.float32, device=self.dev)
        for name, cin, cout in self.specs:
            w, bias = w0[name]
            self.p[name] = dict(
                cin=cin, cout=cout,
                w=torch.tensor(np.asarray(w, np.float32).reshape(27, cout, cin), **f32),
                bias=torch.tensor(np.asarray(bias, np.float32), **f32),
                wf=torch.empty(27 * cout * cin, dtype=torch.bfloat16, device=self.dev),
                wb=torch.empty(27 * cout * cin, dtype=torch.bfloat16, device=self.dev))
            if train:
                self.p[name].update(gw=torch.zeros(27 * cout * cin, **f32),
                                    gb=torch.zeros(cout, **f32))
        # the first convolution's weights on the inference input's channels
        self.p["e1a"].update(
            wf_in=torch.empty(27 * LEVELS[0] * INFER_C, dtype=torch.bfloat16, device=self.dev),
            wb_in=torch.empty(27 * LEVELS[0] * INFER_C, dtype=torch.bfloat16, device=self.dev))
        hw, hb = w0["head"]
        self.p["head"] = dict(w=torch.tensor(np.asarray(hw, np.float32), **f32),
                              bias=torch.tensor(np.asarray(hb, np.float32), **f32))
        self.step_count = 0
        self.record = None  # a dict: backward() keeps every intermediate gradient there
        self.partial = torch.zeros(1024, dtype=torch.float64, device=self.dev)
        self.loss_dev = torch.zeros(1, dtype=torch.float64, device=self.dev)
        if not train:
            self.adam, self.ws, self.ws_bytes = None, None, 0
            self.prep()
            return
        self.p["head"].update(gw=torch.zeros(LEVELS[0], **f32), gb=torch.zeros(1, **f32))
        self.adam = {k: (torch.zeros_like(v["w"]), torch.zeros_like(v["w"]),
                         torch.zeros_like(v["bias"]), torch.zeros_like(v["bias"]))
                     for k, v in self.p.items()}
        # weight-gradient scratch: the largest layer at its resolution
        need = 0
        for name, cin, cout in self.specs:
            s = self._size_of(name)
            nb = C.c_size_t()
            N.check(self.L.vesis_nn_wgrad_workspace(batch, s, s, s, cin, cout, C.byref(nb)),
                    "wgrad workspace")
            need = max(need, nb.value)
        need = max(need, 4 * LEVELS[0] * (batch * size ** 3 // 1024 + 1))  # head sums
        self.ws = torch.empty(need // 4 + 1, **f32)
        self.ws_bytes = need
        self.prep()

    def weights(self):
        """The FP32 master weights, in the form the constructor takes."""
        out = {}
        for name, cin, cout in self.specs:
            q = self.p[name]
            out[name] = (q["w"].cpu().numpy().reshape(27, cout, cin).copy(),
                         q["bias"].cpu().numpy().copy())
        h = self.p["head"]
        out["head"] = (h["w"].cpu().numpy().copy(), h["bias"].cpu().numpy().copy())
        return out

    # ------------------------------------------------------------ helpers
    def _size_of(self, name):
        lvl = int(name[1])
        return self.n >> (lvl - 1)

    def _s(self):
        return C.c_void_p(self.t.cuda.current_stream(self.dev).cuda_stream)

    def _act(self, size, c):
        return self.t.empty((self.b, size, size, size, c), dtype=self.t.bfloat16,
                            device=self.dev)

    def prep(self):
        """BF16 forward and data-gradient weights from the FP32 masters (and
        the first convolution's on the inference input's channels)."""
        for name, cin, cout in self.specs:
            q = self.p[name]
            N.check(self.L.vesis_nn_prep_weights(self._s(), N.ptr(q["w"]), cout, cin,
                                                 N.ptr(q["wf"]), N.ptr(q["wb"])), "prep")
        q = self.p["e1a"]
        w_in = q["w"].reshape(27, q["cout"], q["cin"])[:, :, :INFER_C].contiguous()
        N.check(self.L.vesis_nn_prep_weights(self._s(), N.ptr(w_in), q["cout"], INFER_C,
                                             N.ptr(q["wf_in"]), N.ptr(q["wb_in"])), "prep")

    def conv(self, name, x, relu=True):
        q = self.p[name]
        s = x.shape[1]
        cin, wf = q["cin"], q["wf"]
        if name == "e1a" and x.shape[4] == INFER_C:
            cin, wf = INFER_C, q["wf_in"]
        elif x.shape[4] != cin:
            raise ValueError(f"conv {name}: {x.shape[4]} input channels, expected {cin}")
        y = self._act(s, q["cout"])
        N.check(self.L.vesis_nn_conv3_fwd(self._s(), N.ptr(x), N.ptr(wf), N.ptr(q["bias"]),
                                          N.ptr(y), self.b, s, s, s, cin, q["cout"],
                                          1 if relu else 0), "conv " + name)
        return y

    def conv_upcat(self, name, a, b, relu=True):
        """conv of [up2(a) | b] without forming the upsampled concatenation."""
        q = self.p[name]
        s = b.shape[1]
        y = self._act(s, q["cout"])
        N.check(self.L.vesis_nn_conv3_fwd_upcat(self._s(), N.ptr(a), a.shape[4], N.ptr(b),
                                                b.shape[4], N.ptr(q["wf"]), N.ptr(q["bias"]),
                                                N.ptr(y), self.b, s, s, s, q["cout"],
                                                1 if relu else 0), "conv " + name)
        return y

    def pool(self, x):
        s, c = x.shape[1], x.shape[4]
        y = self._act(s // 2, c)
        N.check(self.L.vesis_nn_pool2(self._s(), N.ptr(x), N.ptr(y), self.b, s, s, s, c, 0),
                "pool")
        return y

    def up(self, x):
        s, c = 2 * x.shape[1], x.shape[4]
        y = self._act(s, c)
        N.check(self.L.vesis_nn_up2(self._s(), N.ptr(x), N.ptr(y), self.b, s, s, s, c, 0), "up")
        return y

    def cat(self, a, b):
        s = a.shape[1]
        y = self._act(s, a.shape[4] + b.shape[4])
        P = self.b * s ** 3
        N.check(self.L.vesis_nn_concat(self._s(), N.ptr(a), a.shape[4], N.ptr(b), b.shape[4],
                                       N.ptr(y), P), "concat")
        return y

    # ------------------------------------------------------------ forward
    def featurize(self, pos4, sigma, q, h, center, out=None, channels=IN_C):
        """Input channels for one molecule (device FP64 arrays) on this grid:
        IN_C for training, INFER_C for inference (forward with keep=False)."""
        x = out if out is not None else self._act(self.n, channels)
        if x.shape[4] != channels:
            raise ValueError("featurize: the output tensor's channels differ from `channels`")
        cen = (C.c_double * 3)(*[float(v) for v in center])
        N.check(self.L.vesis_nn_featurize(self._s(), N.ptr(pos4), N.ptr(sigma), N.ptr(q),
                                          int(sigma.numel()), self.n, float(h),
                                          C.cast(cen, C.c_void_p), channels, N.ptr(x)),
                "featurize")
        return x

    def forward(self, x, keep: bool = True):
        """x: (b, n, n, n, IN_C) BF16, or (b, n, n, n, INFER_C) for
        inference.  Returns logits (b n^3 FP32).  keep: hold the activations
        for backward; without it (inference) the decoder convolutions read
        [up2(deeper) | skip] in place."""
        if not keep:
            return self._infer(x)
        if x.shape[4] != IN_C:
            raise ValueError(f"forward with keep=True takes {IN_C} input channels")
        a = {"x": x}
        a["a1"] = self.conv("e1a", x)
        a["s1"] = self.conv("e1b", a["a1"])
        a["p1"] = self.pool(a["s1"])
        a["a2"] = self.conv("e2a", a["p1"])
        a["s2"] = self.conv("e2b", a["a2"])
        a["p2"] = self.pool(a["s2"])
        a["a3"] = self.conv("e3a", a["p2"])
        a["s3"] = self.conv("e3b", a["a3"])
        a["p3"] = self.pool(a["s3"])
        a["a4"] = self.conv("e4a", a["p3"])
        a["b4"] = self.conv("e4b", a["a4"])
        a["c3"] = self.cat(self.up(a["b4"]), a["s3"])
        a["a5"] = self.conv("d3a", a["c3"])
        a["b5"] = self.conv("d3b", a["a5"])
        a["c2"] = self.cat(self.up(a["b5"]), a["s2"])
        a["a6"] = self.conv("d2a", a["c2"])
        a["b6"] = self.conv("d2b", a["a6"])
        a["c1"] = self.cat(self.up(a["b6"]), a["s1"])
        a["a7"] = self.conv("d1a", a["c1"])
        a["b7"] = self.conv("d1b", a["a7"])
        P = self.b * self.n ** 3
        logits = self.t.empty(P, dtype=self.t.float32, device=self.dev)
        h = self.p["head"]
        N.check(self.L.vesis_nn_head_fwd(self._s(), N.ptr(a["b7"]), N.ptr(h["w"]), N.ptr(h["bias"]),
                                         N.ptr(logits), P, LEVELS[0]), "head")
        self.acts = a
        return logits

    def _infer(self, x):
        def upcat(name, a, b):
            if b.shape[1] >= 16:
                return self.conv_upcat(name, a, b)
            return self.conv(name, self.cat(self.up(a), b))
        s1 = self.conv("e1b", self.conv("e1a", x))
        s2 = self.conv("e2b", self.conv("e2a", self.pool(s1)))
        s3 = self.conv("e3b", self.conv("e3a", self.pool(s2)))
        b4 = self.conv("e4b", self.conv("e4a", self.pool(s3)))
        b5 = self.conv("d3b", upcat("d3a", b4, s3))
        b6 = self.conv("d2b", upcat("d2a", b5, s2))
        b7 = self.conv("d1b", upcat("d1a", b6, s1))
        P = self.b * self.n ** 3
        logits = self.t.empty(P, dtype=self.t.float32, device=self.dev)
        h = self.p["head"]
        N.check(self.L.vesis_nn_head_fwd(self._s(), N.ptr(b7), N.ptr(h["w"]), N.ptr(h["bias"]),
                                         N.ptr(logits), P, LEVELS[0]), "head")
        self.acts = None
        return logits

    # ------------------------------------------------------------ backward
    def _relu_bwd(self, y, dy):
        g = self.t.empty_like(y)
        N.check(self.L.vesis_nn_relu_bwd(self._s(), N.ptr(y), N.ptr(dy), N.ptr(g), y.numel()),
                "relu_bwd")
        return g

    def _conv_bwd(self, name, x, y, dy, need_dx=True):
        """Gradient through y = relu(conv(x)): weight and bias gradients, and
        the gradient at x (unless need_dx is False)."""
        q = self.p[name]
        s = x.shape[1]
        g = self._relu_bwd(y, dy)
        N.check(self.L.vesis_nn_conv3_wgrad(self._s(), N.ptr(x), N.ptr(g), N.ptr(q["gw"]),
                                            N.ptr(q["gb"]), N.ptr(self.ws), self.ws_bytes, self.b,
                                            s, s, s, q["cin"], q["cout"]), "wgrad " + name)
        if not need_dx:
            if self.record is not None:
                self.record[name] = (dy, None)
            return None
        dx = self._act(s, q["cin"])
        N.check(self.L.vesis_nn_conv3_fwd(self._s(), N.ptr(g), N.ptr(q["wb"]), None, N.ptr(dx),
                                          self.b, s, s, s, q["cout"], q["cin"], 0),
                "dgrad " + name)
        if self.record is not None:
            self.record[name] = (dy, dx)
        return dx

    def _split(self, dcat, ca):
        s = dcat.shape[1]
        cb = dcat.shape[4] - ca
        da, db = self._act(s, ca), self._act(s, cb)
        N.check(self.L.vesis_nn_split(self._s(), N.ptr(dcat), ca, cb, N.ptr(da), N.ptr(db), 0,
                                      self.b * s ** 3), "split")
        return da, db

    def _up_bwd(self, dy):
        s, c = dy.shape[1], dy.shape[4]
        dx = self._act(s // 2, c)
        N.check(self.L.vesis_nn_up2(self._s(), N.ptr(dy), N.ptr(dx), self.b, s, s, s, c, 1),
                "up_bwd")
        if self.record is not None:
            self.record["up", s] = (dy, dx)
        return dx

    def _pool_bwd_add(self, dp, dskip):
        """dskip + the adjoint of pooling applied to dp (in place on dskip)."""
        s, c = dskip.shape[1], dskip.shape[4]
        if self.record is not None:
            self.record["pool", s] = (dp, dskip.clone(), dskip)
        t = self._act(s, c)
        N.check(self.L.vesis_nn_pool2(self._s(), N.ptr(dp), N.ptr(t), self.b, s, s, s, c, 1),
                "pool_bwd")
        N.check(self.L.vesis_nn_add(self._s(), N.ptr(dskip), N.ptr(t), N.ptr(dskip),
                                    dskip.numel()), "add")
        return dskip

    def backward(self, dlogit):
        """Gradients of every parameter from dlogit (b n^3 FP32)."""
        a = self.acts
        h = self.p["head"]
        P = self.b * self.n ** 3
        db7 = self.t.empty_like(a["b7"])
        N.check(self.L.vesis_nn_head_bwd(self._s(), N.ptr(dlogit), N.ptr(a["b7"]), N.ptr(h["w"]),
                                         N.ptr(db7), N.ptr(h["gw"]), N.ptr(h["gb"]),
                                         N.ptr(self.ws), self.ws_bytes, P, LEVELS[0]),
                "head_bwd")
        if self.record is not None:
            self.record["head"] = (dlogit, db7)
        c1, c2, c3, _ = LEVELS
        da7 = self._conv_bwd("d1b", a["a7"], a["b7"], db7)
        dc1 = self._conv_bwd("d1a", a["c1"], a["a7"], da7)
        du1, ds1 = self._split(dc1, c2)
        db6 = self._up_bwd(du1)
        da6 = self._conv_bwd("d2b", a["a6"], a["b6"], db6)
        dc2 = self._conv_bwd("d2a", a["c2"], a["a6"], da6)
        du2, ds2 = self._split(dc2, c3)
        db5 = self._up_bwd(du2)
        da5 = self._conv_bwd("d3b", a["a5"], a["b5"], db5)
        dc3 = self._conv_bwd("d3a", a["c3"], a["a5"], da5)
        du3, ds3 = self._split(dc3, LEVELS[3])
        db4 = self._up_bwd(du3)
        da4 = self._conv_bwd("e4b", a["a4"], a["b4"], db4)
        dp3 = self._conv_bwd("e4a", a["p3"], a["a4"], da4)
        ds3 = self._pool_bwd_add(dp3, ds3)
        da3 = self._conv_bwd("e3b", a["a3"], a["s3"], ds3)
        dp2 = self._conv_bwd("e3a", a["p2"], a["a3"], da3)
        ds2 = self._pool_bwd_add(dp2, ds2)
        da2 = self._conv_bwd("e2b", a["a2"], a["s2"], ds2)
        dp1 = self._conv_bwd("e2a", a["p1"], a["a2"], da2)
        ds1 = self._pool_bwd_add(dp1, ds1)
        da1 = self._conv_bwd("e1b", a["a1"], a["s1"], ds1)
        self._conv_bwd("e1a", a["x"], a["a1"], da1, need_dx=False)

    def loss(self, logits, labels, pos_weight: float = 1.0):
        """Mean BCE against labels (device int8, -1 solute): (device loss, dlogit)."""
        P = logits.numel()
        dlogit = self.t.empty_like(logits)
        N.check(self.L.vesis_nn_bce(self._s(), N.ptr(logits), N.ptr(labels), P, float(pos_weight),
                                    N.ptr(dlogit), N.ptr(self.partial), 1024,
                                    N.ptr(self.loss_dev)), "bce")
        return self.loss_dev, dlogit

    def adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step_count += 1
        for k, q in self.p.items():
            m_w, v_w, m_b, v_b = self.adam[k]
            N.check(self.L.vesis_nn_adam(self._s(), N.ptr(q["w"]), N.ptr(q["gw"]), N.ptr(m_w),
                                         N.ptr(v_w), q["w"].numel(), lr, b1, b2, eps,
                                         self.step_count), "adam")
            N.check(self.L.vesis_nn_adam(self._s(), N.ptr(q["bias"]), N.ptr(q["gb"]), N.ptr(m_b),
                                         N.ptr(v_b), q["bias"].numel(), lr, b1, b2, eps,
                                         self.step_count), "adam")
        self.prep()

    def grads(self):
        out = {}
        for name, cin, cout in self.specs:
            q = self.p[name]
            out[name] = (q["gw"].cpu().numpy().reshape(27, cout, cin), q["gb"].cpu().numpy())
        out["head"] = (self.p["head"]["gw"].cpu().numpy(), self.p["head"]["gb"].cpu().numpy())
        return out


def molecule_arrays(w, device):
    """Device FP64 arrays (pos4, sigma, q) of a synth.Workload."""
    import torch
    pos4 = np.zeros((w.natoms, 4))
    pos4[:, :3] = w.xyz
    dd = dict(dtype=torch.float64, device=device)
    return (torch.tensor(pos4, **dd), torch.tensor(np.asarray(w.sigma, np.float64), **dd),
            torch.tensor(np.asarray(w.q, np.float64), **dd))


class Sample:
    """One training molecule on the device: its atoms and the labels the
    relaxation reached from the tight start."""

    def __init__(self, w, labels_host, device):
        import torch
        self.w = w
        self.pos4, self.sigma, self.q = molecule_arrays(w, device)
        self.labels = torch.tensor(np.asarray(labels_host, np.int8), device=device)


def relaxed_labels(workloads, batch: int = 64):
    """Equilibrium labels of each workload from the tight start (the
    relaxation of Step 2, batched), as host int8 arrays, with the sweeps."""
    from .vesis import Batch, Context
    out, sweeps = [], []
    for k in range(0, len(workloads), batch):
        ctxs = []
        for w in workloads[k:k + batch]:
            c = Context(0)
            c.setup(w, precision=32)
            c.init_labels("tight", 1.0)
            ctxs.append(c)
        rc, st = Batch(ctxs).minimize()
        for c, s in zip(ctxs, st):
            out.append(c.labels())
            sweeps.append(s["sweeps"])
            c.close()
    return out, sweeps


def train(model: UNet, samples, steps: int, lr: float = 1e-3, pos_weight: float = 1.0,
          log_every: int = 0, log=print):
    """Adam on the mean BCE, one sample per step, cycling through samples.
    Returns the loss of every step."""
    import torch
    x = model._act(model.n, IN_C)
    losses = []
    for s in range(steps):
        smp = samples[s % len(samples)]
        model.featurize(smp.pos4, smp.sigma, smp.q, smp.w.h, smp.w.center, out=x)
        logits = model.forward(x)
        loss, dlogit = model.loss(logits, smp.labels, pos_weight)
        losses.append(loss.clone())
        model.backward(dlogit)
        model.adam_step(lr)
        if log_every and (s + 1) % log_every == 0:
            log(f"step {s + 1}: loss {float(torch.stack(losses[-log_every:]).mean()):.4f}")
    return [float(v) for v in torch.stack(losses).cpu().numpy().ravel()]


def predict_logits(model: UNet, pos4, sigma, q, h, center):
    x = model.featurize(pos4, sigma, q, h, center, channels=INFER_C)
    return model.forward(x, keep=False)


def warm_start_experiment(n_train: int = 2000, n_test: int = 32, epochs: int = 1,
                          lr: float = 1e-3, seed: int = 0, log=print):
    """Train the network on relaxed labels of n_train molecules (128^3 grid,
    0.05 nm) and compare, on n_test held-out molecules, the relaxation from
    the tight start with the relaxation from the network's labels: sweeps,
    wall time (density, far field and sweeps included; for the learned start
    also featurisation and the network), and the free energy reached.
    Molecule by molecule and batched."""
    import time

    import torch

    import synth
    from .vesis import Batch, Context
    dev = torch.device("cuda")
    t0 = time.perf_counter()
    train_set = synth.warm_start_set(n_train, seed0=5000)
    test_set = synth.warm_start_set(n_test, seed0=9000)
    labels, train_sweeps = relaxed_labels(train_set)
    samples = [Sample(w, lab, dev) for w, lab in zip(train_set, labels)]
    del labels
    t1 = time.perf_counter()
    log(f"training set: {n_train} molecules relaxed in {t1 - t0:.1f} s")
    model = UNet(128, seed=seed)
    losses = train(model, samples, steps=epochs * n_train, lr=lr,
                   log_every=max(1, n_train // 4), log=log)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    log(f"trained {epochs * n_train} steps in {t2 - t1:.1f} s")
    del samples

    ctxs, arrays = [], []
    for w in test_set:
        c = Context(0)
        c.setup(w, precision=32)
        ctxs.append(c)
        arrays.append(molecule_arrays(w, dev))

    def plain(c, w):
        c.set_positions(w.xyz)
        c.init_labels("tight", 1.0)
        return c.minimize()[1]

    def learned(c, w, a):
        c.set_positions(w.xyz)
        logits = predict_logits(model, a[0], a[1], a[2], w.h, w.center)
        c.init_labels_logits(logits)
        return c.minimize()[1]

    rows = []
    for k, (c, w, a) in enumerate(zip(ctxs, test_set, arrays)):
        for rep in range(2):  # the first pass warms up
            torch.cuda.synchronize()
            ta = time.perf_counter()
            sp = plain(c, w)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            gp = c.energy()["total"]
            lab_p = c.labels()
            torch.cuda.synchronize()
            tc = time.perf_counter()
            sl = learned(c, w, a)
            torch.cuda.synchronize()
            td = time.perf_counter()
        gl = c.energy()["total"]
        agree = float((c.labels() == lab_p).mean())
        rows.append(dict(atoms=w.natoms, plain_sweeps=sp["sweeps"], learned_sweeps=sl["sweeps"],
                         plain_flips=sp["flips"], learned_flips=sl["flips"],
                         plain_ms=1e3 * (tb - ta), learned_ms=1e3 * (td - tc),
                         G_plain=gp, G_learned=gl, label_agreement=agree))
    # batched: every test molecule at once; the network's inference either
    # one molecule at a time or as one batch of all of them (a copy of the
    # trained weights in an inference-only model of that batch size)
    b = Batch(ctxs)
    times = {}
    inf = UNet(128, batch=len(test_set), weights=model.weights(), train=False)
    xb = inf._act(128, INFER_C)
    n3 = 128 ** 3
    for rep in range(2):
        for c, w in zip(ctxs, test_set):
            c.set_positions(w.xyz)
            c.init_labels("tight", 1.0)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        rc, stp = b.minimize()
        torch.cuda.synchronize()
        times["plain_batched_ms"] = 1e3 * (time.perf_counter() - ta)
        for c, w in zip(ctxs, test_set):
            c.set_positions(w.xyz)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for c, w, a in zip(ctxs, test_set, arrays):
            c.init_labels_logits(predict_logits(model, a[0], a[1], a[2], w.h, w.center))
        rc, stl = b.minimize()
        torch.cuda.synchronize()
        times["learned_batched_serial_inference_ms"] = 1e3 * (time.perf_counter() - ta)
        for c, w in zip(ctxs, test_set):
            c.set_positions(w.xyz)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for i, (w, a) in enumerate(zip(test_set, arrays)):
            inf.featurize(a[0], a[1], a[2], w.h, w.center, out=xb[i:i + 1], channels=INFER_C)
        logits = inf.forward(xb, keep=False)
        for i, c in enumerate(ctxs):
            c.init_labels_logits(logits[i * n3:(i + 1) * n3])
        rc, stl2 = b.minimize()
        torch.cuda.synchronize()
        times["learned_batched_ms"] = 1e3 * (time.perf_counter() - ta)
        del logits
        assert [s_["sweeps"] for s_ in stl2] == [s_["sweeps"] for s_ in stl]
    for c in ctxs:
        c.close()
    dG = [abs(r["G_learned"] - r["G_plain"]) / abs(r["G_plain"]) for r in rows]
    return {
        "train_molecules": n_train, "test_molecules": n_test, "epochs": epochs, "grid": 128,
        "train_relax_s": t1 - t0, "train_s": t2 - t1,
        "train_loss_first": float(np.mean(losses[:50])), "train_loss_last": float(np.mean(losses[-50:])),
        "plain_sweeps_mean": float(np.mean([r["plain_sweeps"] for r in rows])),
        "learned_sweeps_mean": float(np.mean([r["learned_sweeps"] for r in rows])),
        "plain_ms_mean": float(np.mean([r["plain_ms"] for r in rows])),
        "learned_ms_mean": float(np.mean([r["learned_ms"] for r in rows])),
        "max_rel_dG": float(max(dG)), "median_rel_dG": float(np.median(dG)),
        "learned_G_lower_or_equal": int(sum(r["G_learned"] <= r["G_plain"] for r in rows)),
        "label_agreement_mean": float(np.mean([r["label_agreement"] for r in rows])),
        "plain_batched_sweeps_max": max(s["sweeps"] for s in stp),
        "learned_batched_sweeps_max": max(s["sweeps"] for s in stl),
        **times, "rows": rows}


def conv_flops(n: int, batch: int = 1, in_c: int = IN_C) -> float:
    """Multiply-add work (2 flops each) of the network's 3x3x3 convolutions at
    grid n: 27 cin cout per position at each layer's resolution, the first
    layer reading in_c channels (INFER_C for inference)."""
    total = 0.0
    for name, cin, cout in layer_specs():
        s = n >> (int(name[1]) - 1)
        if name == "e1a":
            cin = in_c
        total += 2.0 * 27 * cin * cout * batch * s ** 3
    return total


def inference_timing(n: int = 128, batch: int = 16, reps: int = 5, seed: int = 0):
    """Device time of the inference forward pass (keep=False) of an
    inference-only network (initial weights) on random BF16 input of `batch`
    grids of n^3 cells and INFER_C channels; returns ms per batch, ms per
    molecule and the convolutions' TFLOP/s."""
    import time

    import torch
    m = UNet(n, batch=batch, seed=seed, train=False)
    x = m._act(n, INFER_C)
    g = torch.Generator(device=m.dev).manual_seed(seed)
    x.copy_(torch.rand(x.shape, generator=g, device=m.dev).to(torch.bfloat16))
    m.forward(x, keep=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        m.forward(x, keep=False)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    return {"grid": n, "batch": batch, "ms_per_batch": ms, "ms_per_molecule": ms / batch,
            "conv_tflops": conv_flops(n, batch, INFER_C) / (ms * 1e-3) / 1e12,
            "conv_flop_per_molecule": conv_flops(n, 1, INFER_C)}


if __name__ == "__main__":
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="train and evaluate the learned warm start")
    ap.add_argument("--infer-only", action="store_true",
                    help="only time the inference forward pass (--grid, --batch, --reps)")
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--test", type=int, default=32)
    ap.add_argument("--epochs", type=int, default=1)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    if args.infer_only:
        print(json.dumps(inference_timing(args.grid, args.batch, args.reps)), flush=True)
        sys.exit(0)
    res = warm_start_experiment(args.train, args.test, args.epochs, args.lr,
                                log=lambda *a: print(*a, file=sys.stderr, flush=True))
    text = json.dumps(res)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text + "\n")
    print(json.dumps({k: v for k, v in res.items() if k != "rows"}), flush=True)
