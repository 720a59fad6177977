"""Pins of the FP64 reference network (oracle/unet.py) on the CPU: its
convolution against the definition written as loops, its pooling and
upsampling against their definitions, and its autograd gradients against
central differences of its loss."""
import numpy as np

import synth
from oracle import unet


def _rng(seed):
    return np.random.default_rng(seed)


def test_oracle_conv_is_the_defining_sum():
    """Y[p][co] = sum_{tap, ci} X[p + off(tap)][ci] W[tap][co][ci], zero
    padding, tap = 9 (dz+1) + 3 (dy+1) + (dx+1)."""
    import torch
    r = _rng(1)
    n, cin, cout = 4, 2, 3
    x = r.standard_normal((1, n, n, n, cin))
    w = r.standard_normal((27, cout, cin))
    b = r.standard_normal(cout)
    xt = torch.as_tensor(x).permute(0, 4, 1, 2, 3)
    y = unet.conv(xt, unet.to_torch_weight(w), torch.as_tensor(b), relu=False)
    y = y.permute(0, 2, 3, 4, 1).numpy()
    ref = np.zeros((1, n, n, n, cout))
    for z in range(n):
        for yy in range(n):
            for xx in range(n):
                acc = b.copy()
                for tap in range(27):
                    dz, dy, dx = tap // 9 - 1, (tap // 3) % 3 - 1, tap % 3 - 1
                    zz, y2, x2 = z + dz, yy + dy, xx + dx
                    if 0 <= zz < n and 0 <= y2 < n and 0 <= x2 < n:
                        acc += w[tap] @ x[0, zz, y2, x2]
                ref[0, z, yy, xx] = acc
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)


def test_oracle_pool_and_upsample_are_their_definitions():
    import torch
    import torch.nn.functional as F
    r = _rng(2)
    x = r.standard_normal((1, 3, 4, 6, 8))  # (b, c, z, y, x)
    p = F.avg_pool3d(torch.as_tensor(x), 2).numpy()
    ref = x.reshape(1, 3, 2, 2, 3, 2, 4, 2).mean(axis=(3, 5, 7))
    np.testing.assert_allclose(p, ref, rtol=1e-14)
    u = F.interpolate(torch.as_tensor(x), scale_factor=2, mode="nearest").numpy()
    zi, yi, xi = np.meshgrid(np.arange(8) // 2, np.arange(12) // 2, np.arange(16) // 2,
                             indexing="ij")
    np.testing.assert_array_equal(u, x[:, :, zi, yi, xi])


def test_oracle_gradients_match_central_differences():
    """d loss / d w of the oracle's autograd against central differences of
    its own forward, for weights in the first, bottleneck, decoder and head
    layers (8^3 grid, random input and labels)."""
    r = _rng(3)
    w = synth.conv_weights(unet.SPECS, 32, seed=7)
    x = r.standard_normal((1, 8, 8, 8, 32))
    lab = np.where(r.random(8 ** 3) < 0.3, -1, 1).astype(np.int8)
    out = unet.forward(w, x, lab, pos_weight=2.0, grads=True)
    g = out["grads"]
    checks = [("e1a", (4, 3, 1)), ("e4b", (13, 7, 200)), ("d3a", (0, 5, 300)),
              ("d1b", (26, 31, 2)), ("head", (5,))]
    eps = 1e-6
    for name, idx in checks:
        wp = {k: (v[0].astype(np.float64).copy(), v[1].astype(np.float64).copy())
              for k, v in w.items()}
        wm = {k: (v[0].astype(np.float64).copy(), v[1].astype(np.float64).copy())
              for k, v in w.items()}
        wp[name][0][idx] += eps
        wm[name][0][idx] -= eps
        fd = (unet.forward(wp, x, lab, 2.0)["loss"] - unet.forward(wm, x, lab, 2.0)["loss"]) / (2 * eps)
        an = g[name][0][idx]
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-4), (name, idx, fd, an)
