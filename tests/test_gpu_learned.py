"""The learned warm start on the GPU: each layer and the whole network
against the FP64 reference network of oracle/unet.py, training, and the
labels it starts the relaxation from."""
import numpy as np
import pytest

import synth
from helpers import check_labels, log

pytestmark = pytest.mark.gpu


def _bf(a):
    """Round to BF16 and back (the GPU's storage precision)."""
    import torch
    return torch.tensor(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _dev_bf16(a):
    import torch
    return torch.tensor(np.asarray(a, np.float32), device="cuda").to(torch.bfloat16).contiguous()


def _stream():
    import ctypes
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _rel(a, b):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("n,ca,cb,cout,relu", [(16, 64, 32, 32, 1), (20, 32, 16, 64, 0),
                                               (32, 256, 128, 128, 1), (36, 64, 32, 32, 1)])
def test_conv_upcat_equals_conv_of_the_concatenated_upsample(n, ca, cb, cout, relu):
    """The decoder convolution that reads [up2(a) | b] in place equals, bit
    for bit, the convolution of the materialised concatenation (both
    output-channel tilings, grids ragged against the 32 x 4 x MT tiles)."""
    import torch

    from paper_2208_05524_amd import nn
    r = np.random.default_rng(n * 1000 + ca + cb)
    a = _dev_bf16(r.standard_normal((1, n // 2, n // 2, n // 2, ca)))
    b = _dev_bf16(r.standard_normal((1, n, n, n, cb)))
    w = _dev_bf16(0.1 * r.standard_normal((27, cout, ca + cb)))
    bias = torch.tensor(r.standard_normal(cout).astype(np.float32), device="cuda")
    L = nn.lib()
    up = torch.empty((1, n, n, n, ca), dtype=torch.bfloat16, device="cuda")
    cat = torch.empty((1, n, n, n, ca + cb), dtype=torch.bfloat16, device="cuda")
    y0 = torch.empty((1, n, n, n, cout), dtype=torch.bfloat16, device="cuda")
    y1 = torch.full((1, n, n, n, cout), float("nan"), dtype=torch.bfloat16, device="cuda")
    nn.check(L.vesis_nn_up2(_stream(), nn.ptr(a), nn.ptr(up), 1, n, n, n, ca, 0), "up")
    nn.check(L.vesis_nn_concat(_stream(), nn.ptr(up), ca, nn.ptr(b), cb, nn.ptr(cat), n ** 3), "cat")
    nn.check(L.vesis_nn_conv3_fwd(_stream(), nn.ptr(cat), nn.ptr(w), nn.ptr(bias), nn.ptr(y0), 1,
                                  n, n, n, ca + cb, cout, relu), "conv")
    nn.check(L.vesis_nn_conv3_fwd_upcat(_stream(), nn.ptr(a), ca, nn.ptr(b), cb, nn.ptr(w),
                                        nn.ptr(bias), nn.ptr(y1), 1, n, n, n, cout, relu), "upcat")
    torch.cuda.synchronize()
    assert torch.equal(y0.view(torch.int16), y1.view(torch.int16))


def test_inference_forward_equals_training_forward():
    """The network's inference pass (decoder inputs read in place) gives the
    training forward's logits bit for bit (64^3: every decoder level >= 16)."""
    import torch

    from paper_2208_05524_amd.learned import IN_C, UNet
    m = UNet(64, seed=3)
    r = np.random.default_rng(7)
    x = _dev_bf16(np.abs(r.standard_normal((1, 64, 64, 64, IN_C))))
    l0 = m.forward(x).clone()
    l1 = m.forward(x, keep=False)
    torch.cuda.synchronize()
    assert torch.equal(l0, l1)


def test_batched_inference_equals_one_molecule_at_a_time():
    """An inference-only model of batch 3 built from another model's weights
    gives, for each sample, the logits that model gives for it alone, bit for
    bit (32^3: the decoder's 16^3 level reads its inputs in place)."""
    import torch

    from paper_2208_05524_amd.learned import IN_C, UNet
    m = UNet(32, seed=4)
    r = np.random.default_rng(8)
    x = _dev_bf16(np.abs(r.standard_normal((3, 32, 32, 32, IN_C))))
    one = [m.forward(x[i:i + 1].contiguous(), keep=False).clone() for i in range(3)]
    inf = UNet(32, batch=3, weights=m.weights(), train=False)
    assert inf.adam is None and "gw" not in inf.p["e1a"]
    lb = inf.forward(x, keep=False)
    torch.cuda.synchronize()
    n3 = 32 ** 3
    for i in range(3):
        assert torch.equal(lb[i * n3:(i + 1) * n3], one[i]), i


@pytest.mark.parametrize("n,cin,cout,relu", [(8, 32, 64, 1), (6, 16, 32, 0), (5, 96, 32, 1),
                                             (16, 32, 64, 1), (20, 32, 32, 1), (18, 16, 64, 0),
                                             (24, 96, 32, 1)])
def test_conv_forward_matches_reference(n, cin, cout, relu):
    """Both kernels (grids narrower than 16 cells take the direct one, wider
    ones the LDS-tiled one), ragged sizes against their tiles (128 positions;
    32 x 4 x MT), both output-channel tilings, with and without ReLU: every
    output within BF16 rounding of the FP64 convolution of the same BF16
    inputs."""
    import torch

    from oracle import unet
    from paper_2208_05524_amd import nn
    r = np.random.default_rng(n * 100 + cin)
    x = _bf(r.standard_normal((1, n, n, n, cin)))
    w = _bf(0.1 * r.standard_normal((27, cout, cin)))
    b = r.standard_normal(cout).astype(np.float32)
    ref = unet.conv(torch.as_tensor(x).permute(0, 4, 1, 2, 3), unet.to_torch_weight(w),
                    torch.as_tensor(b.astype(np.float64)), relu=bool(relu))
    ref = ref.permute(0, 2, 3, 4, 1).numpy()
    L = nn.lib()
    xd, wd = _dev_bf16(x), _dev_bf16(w)
    bd = torch.tensor(b, device="cuda")
    yd = torch.empty((1, n, n, n, cout), dtype=torch.bfloat16, device="cuda")
    nn.check(L.vesis_nn_conv3_fwd(_stream(), nn.ptr(xd), nn.ptr(wd), nn.ptr(bd), nn.ptr(yd), 1, n,
                                  n, n, cin, cout, relu), "conv")
    y = yd.float().cpu().numpy()
    err = np.abs(y - ref)
    lim = 2.0 ** -8 * np.abs(ref) + 1e-5 * np.abs(ref).max()
    log("conv max err/lim", float((err / lim).max()))
    assert np.all(err <= lim)


@pytest.mark.parametrize("d,h,w,cin,cout", [(128, 6, 36, 16, 64), (256, 6, 36, 16, 32),
                                             (24, 6, 36, 32, 64)])
def test_conv_forward_tilings_match_reference(d, h, w, cin, cout):
    """The three LDS-tiled kernels (the prefetching one for 64 or more output
    channels, MT = 4 for 32, and MT = 1 for layers with fewer workgroups
    than CUs), chosen by the grid's size and channels: long
    grids ragged in x and y against the 32 x 4 x MT tiles, every output
    within BF16 rounding of the FP64 convolution of the same inputs."""
    import torch

    from oracle import unet
    from paper_2208_05524_amd import nn
    r = np.random.default_rng(d + cout)
    x = _bf(r.standard_normal((1, d, h, w, cin)))
    wt = _bf(0.1 * r.standard_normal((27, cout, cin)))
    b = r.standard_normal(cout).astype(np.float32)
    ref = unet.conv(torch.as_tensor(x).permute(0, 4, 1, 2, 3), unet.to_torch_weight(wt),
                    torch.as_tensor(b.astype(np.float64)), relu=True)
    ref = ref.permute(0, 2, 3, 4, 1).numpy()
    L = nn.lib()
    xd, wd = _dev_bf16(x), _dev_bf16(wt)
    bd = torch.tensor(b, device="cuda")
    yd = torch.empty((1, d, h, w, cout), dtype=torch.bfloat16, device="cuda")
    nn.check(L.vesis_nn_conv3_fwd(_stream(), nn.ptr(xd), nn.ptr(wd), nn.ptr(bd), nn.ptr(yd), 1, d,
                                  h, w, cin, cout, 1), "conv")
    y = yd.float().cpu().numpy()
    err = np.abs(y - ref)
    lim = 2.0 ** -8 * np.abs(ref) + 1e-5 * np.abs(ref).max()
    log("conv tiling", (d, h, w, cin, cout), "max err/lim", float((err / lim).max()))
    assert np.all(err <= lim)


def test_conv_gradients_match_reference():
    """Data gradient (flipped, transposed weights through the forward
    kernel) within BF16 rounding, weight and bias gradients (FP32 sums of
    exact BF16 products) within 1e-5, against FP64 autograd."""
    import torch

    from oracle import unet
    from paper_2208_05524_amd import nn
    r = np.random.default_rng(11)
    n, cin, cout = 20, 64, 32
    x = _bf(r.standard_normal((1, n, n, n, cin)))
    w = 0.1 * r.standard_normal((27, cout, cin)).astype(np.float32)
    dy = _bf(r.standard_normal((1, n, n, n, cout)))
    xt = torch.as_tensor(x).permute(0, 4, 1, 2, 3).requires_grad_(True)
    wt = unet.to_torch_weight(_bf(w)).requires_grad_(True)
    bt = torch.zeros(cout, dtype=torch.float64, requires_grad=True)
    y = unet.conv(xt, wt, bt, relu=False)
    y.backward(torch.as_tensor(dy).permute(0, 4, 1, 2, 3))
    L = nn.lib()
    w32 = torch.tensor(w, device="cuda")
    wf = torch.empty(w.size, dtype=torch.bfloat16, device="cuda")
    wb = torch.empty(w.size, dtype=torch.bfloat16, device="cuda")
    nn.check(L.vesis_nn_prep_weights(_stream(), nn.ptr(w32), cout, cin, nn.ptr(wf), nn.ptr(wb)),
             "prep")
    dyd, xd = _dev_bf16(dy), _dev_bf16(x)
    dxd = torch.empty((1, n, n, n, cin), dtype=torch.bfloat16, device="cuda")
    nn.check(L.vesis_nn_conv3_fwd(_stream(), nn.ptr(dyd), nn.ptr(wb), None, nn.ptr(dxd), 1, n, n,
                                  n, cout, cin, 0), "dgrad")
    dx_ref = xt.grad.permute(0, 2, 3, 4, 1).numpy()
    err = np.abs(dxd.float().cpu().numpy() - dx_ref)
    assert np.all(err <= 2.0 ** -8 * np.abs(dx_ref) + 1e-5 * np.abs(dx_ref).max())
    import ctypes
    nb = ctypes.c_size_t()
    nn.check(L.vesis_nn_wgrad_workspace(1, n, n, n, cin, cout, ctypes.byref(nb)), "ws")
    ws = torch.empty(nb.value // 4 + 1, dtype=torch.float32, device="cuda")
    dw = torch.empty(w.size, dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    nn.check(L.vesis_nn_conv3_wgrad(_stream(), nn.ptr(xd), nn.ptr(dyd), nn.ptr(dw), nn.ptr(db),
                                    nn.ptr(ws), nb.value, 1, n, n, n, cin, cout), "wgrad")
    dw_ref = unet.from_torch_weight(wt.grad)
    assert _rel(dw.cpu().numpy().reshape(27, cout, cin), dw_ref) < 1e-5
    assert _rel(db.cpu().numpy(), bt.grad.numpy()) < 1e-5


def test_network_forward_and_gradients_match_reference():
    """The whole U-Net (16^3, random input and labels): logits and every
    parameter gradient against the FP64 network with the same BF16-rounded
    weights.  BF16 activations (8-bit significand) through some 30 rounded
    layers of forward and backward bound the agreement: 2 % on logits,
    10 % on gradients (relative L2)."""
    import torch

    from oracle import unet
    from paper_2208_05524_amd.learned import UNet, init_weights
    n = 16
    w = init_weights(seed=3)
    wr = {k: ((_bf(v[0]) if k != "head" else v[0]), v[1]) for k, v in w.items()}
    r = np.random.default_rng(5)
    x = _bf(np.abs(r.standard_normal((1, n, n, n, 32))))
    lab = np.where(r.random(n ** 3) < 0.25, -1, 1).astype(np.int8)
    ref = unet.forward(wr, x, lab, pos_weight=2.0, grads=True)
    m = UNet(n, weights=w)
    logits = m.forward(_dev_bf16(x))
    loss, dlogit = m.loss(logits, torch.tensor(lab, device="cuda"), 2.0)
    m.backward(dlogit)
    g = m.grads()
    rl = _rel(logits.cpu().numpy(), ref["logits"])
    log("logits rel", rl, "loss", float(loss), ref["loss"])
    assert rl < 2e-2
    assert abs(float(loss) - ref["loss"]) < 1e-2 * abs(ref["loss"])
    worst = 0.0
    for k in g:
        e = max(_rel(g[k][0], ref["grads"][k][0]), _rel(g[k][1], ref["grads"][k][1])
                if np.abs(ref["grads"][k][1]).max() > 0 else 0.0)
        log("grad", k, e)
        worst = max(worst, e)
    assert worst < 1e-1


def test_featurize_matches_definition():
    import torch

    from paper_2208_05524_amd.learned import UNet, molecule_arrays
    w = synth.random_small(16, 40, seed=61, h=0.08)
    m = UNet(16)
    pos4, sig, q = molecule_arrays(w, torch.device("cuda"))
    x = m.featurize(pos4, sig, q, w.h, w.center).float().cpu().numpy().reshape(16, 16, 16, 32)
    L = 16 * w.h / 2
    c = -L + (np.arange(16) + 0.5) * w.h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    d0 = np.zeros((16, 16, 16))
    d1 = np.zeros((16, 16, 16))
    for a in range(w.natoms):
        s = 0.5 * w.sigma[a]
        r2 = (X - w.xyz[a, 0]) ** 2 + (Y - w.xyz[a, 1]) ** 2 + (Z - w.xyz[a, 2]) ** 2
        e = np.where(r2 < 16 * s * s, np.exp(-r2 / (2 * s * s)), 0.0)
        d0 += e
        d1 += w.q[a] * e
    assert np.abs(x[..., 0] - d0).max() <= 1e-2 * np.abs(d0).max()
    assert np.abs(x[..., 1] - d1).max() <= 1e-2 * np.abs(d1).max()
    assert np.all(x[..., 2:] == 0)


def test_labels_from_logits():
    import torch

    from helpers import gpu_context
    w = synth.random_small(36, 30, seed=62, h=0.06)
    ctx = gpu_context(w)
    r = np.random.default_rng(7)
    logits = r.standard_normal(36 ** 3).astype(np.float32)
    ctx.init_labels_logits(torch.tensor(logits, device="cuda"))
    assert np.array_equal(ctx.labels(), np.where(logits > 0, -1, 1).astype(np.int8))


def test_training_lowers_the_loss_and_the_warm_start_is_relaxed_exactly():
    """A short training on a few relaxed molecules (32^3) lowers the loss;
    the relaxation from the network's labels reaches a local minimum whose
    labels and energy the oracle's colour schedule reproduces from the same
    start."""
    import torch

    from helpers import gpu_context, oracle_system
    from paper_2208_05524_amd.learned import (Sample, UNet, predict_logits, relaxed_labels,
                                              train)
    ws = [synth.random_small(32, 60, seed=70 + k, h=0.07) for k in range(4)]
    labels, _ = relaxed_labels(ws)
    samples = [Sample(w, lab, torch.device("cuda")) for w, lab in zip(ws, labels)]
    m = UNet(32, seed=1)
    losses = train(m, samples, steps=80, lr=2e-3)
    log("loss first/last", np.mean(losses[:8]), np.mean(losses[-8:]))
    assert np.mean(losses[-8:]) < 0.7 * np.mean(losses[:8])
    w = ws[0]
    smp = samples[0]
    logits = predict_logits(m, smp.pos4, smp.sigma, smp.q, w.h, w.center)
    ctx = gpu_context(w)
    ctx.init_labels_logits(logits)
    start = ctx.labels()
    rc, st = ctx.minimize()
    assert rc == 0
    s = oracle_system(w)
    ulj, ucfa = s.density_grid()
    far = s.far_field()
    phi = start.copy()
    e0 = s.energy(phi, ulj, ucfa, far)["total"]
    _, ost, ties, _ = s.minimize_colour(phi, ulj + ucfa, tie_tol=1e-9 * abs(e0))
    log("warm start sweeps gpu", st["sweeps"], "oracle", ost["sweeps"], "ties", len(ties))
    assert ost["ties"] == len(ties)
    check_labels(ctx.labels(), phi, ties, st, ost, what="warm start")
    e = ctx.energy()["total"]
    assert abs(e - s.energy(phi, ulj, ucfa, far)["total"]) <= 1e-6 * abs(e)
