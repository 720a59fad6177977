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


def test_bf16_rounding_is_round_to_nearest_even():
    """The BF16-storage mode's rounding: 8 significant bits, halfway cases to
    the even neighbour, other values to the nearest, signs symmetric."""
    import torch
    v = torch.tensor([1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, 1 + 2 ** -9,
                      -(1 + 3 * 2 ** -8), 3.0 * 2 ** -100, 255.5, 257.0], dtype=torch.float64)
    want = [1.0, 1 + 2 ** -6, 1 + 2 ** -7, 1.0, -(1 + 2 ** -6), 3.0 * 2 ** -100, 256.0, 256.0]
    assert unet.bf16(v).tolist() == want


def test_written_out_backward_equals_autograd_without_rounding():
    """The BF16-storage mode's layer-by-layer backward pass, with rounding
    off, equals autograd's gradients of the plain float64 network (and the
    same logits and loss): the chain rule is written out correctly."""
    r = _rng(4)
    w = synth.conv_weights(unet.SPECS, 32, seed=9)
    x = r.standard_normal((1, 8, 8, 8, 32))
    lab = np.where(r.random(8 ** 3) < 0.3, -1, 1).astype(np.int8)
    ref = unet.forward(w, x, lab, pos_weight=2.0, grads=True)
    got = unet.forward_backward_bf16(w, x, lab, pos_weight=2.0, rounding=False)
    np.testing.assert_allclose(got["logits"], ref["logits"], rtol=1e-12, atol=1e-12)
    assert abs(got["loss"] - ref["loss"]) <= 1e-12 * abs(ref["loss"])
    for k, (gw, gb) in ref["grads"].items():
        sw = np.abs(gw).max()
        np.testing.assert_allclose(got["grads"][k][0], gw, rtol=1e-9, atol=1e-11 * sw, err_msg=k)
        np.testing.assert_allclose(got["grads"][k][1], gb, rtol=1e-9,
                                   atol=1e-11 * max(np.abs(gb).max(), 1e-300), err_msg=k)


def test_bf16_storage_mode_rounds_what_it_stores():
    """With rounding on, the stored tensors are BF16 values and the result
    differs from the unrounded network by BF16-sized amounts only."""
    r = _rng(6)
    w = synth.conv_weights(unet.SPECS, 32, seed=10)
    x = unet.bf16(__import__("torch").as_tensor(np.abs(r.standard_normal((1, 8, 8, 8, 32))))).numpy()
    lab = np.where(r.random(8 ** 3) < 0.3, -1, 1).astype(np.int8)
    exact = unet.forward_backward_bf16(w, x, lab, 2.0, rounding=False)
    rnd = unet.forward_backward_bf16(w, x, lab, 2.0, rounding=True)
    rel = np.linalg.norm(rnd["logits"] - exact["logits"]) / np.linalg.norm(exact["logits"])
    assert 1e-5 < rel < 5e-2
