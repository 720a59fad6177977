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


@pytest.mark.parametrize("n,batch", [(64, 2), (16, 1)])
def test_inference_on_the_featurised_chunk_equals_the_full_input(n, batch):
    """Inference reads the featurised input as one 16-channel chunk (only
    channels 0 and 1 are nonzero) with the first convolution's weights on
    those channels: the logits equal those from the 32-channel input bit for
    bit, for weights with nonzero biases, through the z-reuse kernel (64^3,
    batch 2) and the one-layer-per-workgroup kernel (16^3)."""
    import torch

    from paper_2208_05524_amd.learned import IN_C, INFER_C, UNet, molecule_arrays
    rng = np.random.default_rng(11)
    w0 = {}
    m0 = UNet(n, seed=12)
    for k, (wk, bk) in m0.weights().items():
        w0[k] = (wk, (0.05 * rng.standard_normal(bk.shape)).astype(np.float32))
    m = UNet(n, batch=batch, weights=w0, train=False)
    ws = [synth.random_small(n, 30 + 20 * i, seed=71 + i, h=0.1) for i in range(batch)]
    x32 = m._act(n, IN_C)
    x16 = m._act(n, INFER_C)
    for i, w in enumerate(ws):
        pos4, sig, q = molecule_arrays(w, torch.device("cuda"))
        m.featurize(pos4, sig, q, w.h, w.center, out=x32[i:i + 1])
        m.featurize(pos4, sig, q, w.h, w.center, out=x16[i:i + 1], channels=INFER_C)
    torch.cuda.synchronize()
    assert torch.equal(x32[..., :INFER_C], x16)
    l32 = m.forward(x32, keep=False).clone()
    l16 = m.forward(x16, keep=False)
    torch.cuda.synchronize()
    assert torch.equal(l32, l16)
    assert float(l32.std()) > 0


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
    """Both LDS-tiled kernels (the z-reuse kernel for layers of 256 or more
    4-layer workgroups, with one or two output-channel tiles, and MT = 1
    below that), chosen by the grid's size: long grids ragged in x and y
    against the 32 x 4 x MT tiles, every output within BF16 rounding of the
    FP64 convolution of the same inputs."""
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


@pytest.mark.parametrize("n,d,h,w,cin,cout,relu", [(3, 42, 18, 40, 48, 32, 0),
                                                    (2, 21, 9, 70, 32, 96, 1),
                                                    (2, 41, 14, 66, 80, 32, 0)])
def test_conv_zreuse_batched_ragged_matches_reference(n, d, h, w, cin, cout, relu):
    """The z-reuse kernel on a batch of molecules (per-molecule offsets),
    ragged in every axis against its 32 x 4 x 4 and 32 x 4 x 8 tiles (z
    too), three and five chunks of input channels (prefetch across chunks),
    one and three output-channel tiles, with and without ReLU."""
    import torch

    from oracle import unet
    from paper_2208_05524_amd import nn
    r = np.random.default_rng(n * 1000 + d + cout)
    x = _bf(r.standard_normal((n, d, h, w, cin)))
    wt = _bf(0.1 * r.standard_normal((27, cout, cin)))
    b = r.standard_normal(cout).astype(np.float32)
    ref = unet.conv(torch.as_tensor(x).permute(0, 4, 1, 2, 3), unet.to_torch_weight(wt),
                    torch.as_tensor(b.astype(np.float64)), relu=bool(relu))
    ref = ref.permute(0, 2, 3, 4, 1).numpy()
    L = nn.lib()
    xd, wd = _dev_bf16(x), _dev_bf16(wt)
    bd = torch.tensor(b, device="cuda")
    yd = torch.full((n, d, h, w, cout), float("nan"), dtype=torch.bfloat16, device="cuda")
    nn.check(L.vesis_nn_conv3_fwd(_stream(), nn.ptr(xd), nn.ptr(wd), nn.ptr(bd), nn.ptr(yd), n, d,
                                  h, w, cin, cout, relu), "conv")
    y = yd.float().cpu().numpy()
    err = np.abs(y - ref)
    lim = 2.0 ** -8 * np.abs(ref) + 1e-5 * np.abs(ref).max()
    log("conv z-reuse", (n, d, h, w, cin, cout, relu), "max err/lim", float((err / lim).max()))
    assert np.all(err <= lim)


def test_conv_zreuse_upcat_batched_equals_concatenation():
    """The z-reuse kernel reading [up2(a) | b] in place on a batch of two
    ragged grids gives the convolution of the materialised concatenation
    bit for bit."""
    import torch

    from paper_2208_05524_amd import nn
    n, d, h, w, ca, cb, cout = 2, 26, 20, 36, 32, 16, 64
    r = np.random.default_rng(77)
    a = _dev_bf16(r.standard_normal((n, d // 2, h // 2, w // 2, ca)))
    b = _dev_bf16(r.standard_normal((n, d, h, w, cb)))
    wt = _dev_bf16(0.1 * r.standard_normal((27, cout, ca + cb)))
    bias = torch.tensor(r.standard_normal(cout).astype(np.float32), device="cuda")
    L = nn.lib()
    P = d * h * w
    up = torch.empty((n, d, h, w, ca), dtype=torch.bfloat16, device="cuda")
    cat = torch.empty((n, d, h, w, ca + cb), dtype=torch.bfloat16, device="cuda")
    y0 = torch.empty((n, d, h, w, cout), dtype=torch.bfloat16, device="cuda")
    y1 = torch.full((n, d, h, w, cout), float("nan"), dtype=torch.bfloat16, device="cuda")
    nn.check(L.vesis_nn_up2(_stream(), nn.ptr(a), nn.ptr(up), n, d, h, w, ca, 0), "up")
    nn.check(L.vesis_nn_concat(_stream(), nn.ptr(up), ca, nn.ptr(b), cb, nn.ptr(cat), n * P), "cat")
    nn.check(L.vesis_nn_conv3_fwd(_stream(), nn.ptr(cat), nn.ptr(wt), nn.ptr(bias), nn.ptr(y0), n,
                                  d, h, w, ca + cb, cout, 1), "conv")
    nn.check(L.vesis_nn_conv3_fwd_upcat(_stream(), nn.ptr(a), ca, nn.ptr(b), cb, nn.ptr(wt),
                                        nn.ptr(bias), nn.ptr(y1), n, d, h, w, cout, 1), "upcat")
    torch.cuda.synchronize()
    assert torch.equal(y0.view(torch.int16), y1.view(torch.int16))


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


def _stored_close(got, ref, what, max_frac=2e-3):
    """A BF16 tensor the GPU stored against the reference layer's stored
    value from the same inputs: equal except where the FP32 and FP64 sums
    fall on different sides of a BF16 rounding boundary (a small fraction),
    and there by at most one BF16 step."""
    got = np.asarray(got, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    d = got != ref
    frac = float(d.mean())
    # one BF16 step of the value, or (a ReLU whose input sits at zero within
    # the sums' rounding) a difference negligible against the tensor
    floor = 1e-6 * np.abs(ref).max()
    step = np.abs(got[d] - ref[d]) / np.maximum(np.abs(ref[d]), floor / 2.0 ** -7 + 1e-300)
    log(f"{what}: {d.sum()} of {d.size} differ, largest {step.max() if d.any() else 0.0:.2e}")
    assert frac <= max_frac, (what, frac)
    assert not d.any() or step.max() <= 2.0 ** -7, (what, step.max())


def test_network_layers_match_the_bf16_storage_reference():
    """Every layer of the whole U-Net (16^3, random input and labels), forward
    and backward, against the reference layer of oracle/unet.py's BF16-storage
    mode fed with the GPU's own inputs to that layer: stored BF16 tensors
    equal up to rare one-step rounding differences, logits within 1e-6,
    weight and bias gradients within 1e-5 (relative L2).  End to end the
    two networks drift apart by about 1 % (each rare one-step difference
    shifts later sums across other rounding boundaries), which the
    comparison with the FP64 network above bounds."""
    import torch

    from oracle import unet
    from paper_2208_05524_amd.learned import UNet, init_weights
    n = 16
    w = init_weights(seed=3)
    r = np.random.default_rng(5)
    x = _bf(np.abs(r.standard_normal((1, n, n, n, 32))))
    lab = np.where(r.random(n ** 3) < 0.25, -1, 1).astype(np.int8)
    m = UNet(n, weights=w)
    m.record = {}
    xd = _dev_bf16(x)
    labd = torch.tensor(lab, device="cuda")
    logits = m.forward(xd)
    loss, dlogit = m.loss(logits, labd, 2.0)
    m.backward(dlogit)
    g = m.grads()

    def T(t):  # device channels-last -> float64 (b, c, z, y, x)
        return torch.as_tensor(t.double().cpu().numpy()).permute(0, 4, 1, 2, 3).contiguous()

    A = {k: T(v) for k, v in m.acts.items()}
    W = {name: (unet.bf16(unet.to_torch_weight(w[name][0])),
                torch.as_tensor(np.asarray(w[name][1], np.float64))) for name, _, _ in unet.SPECS}
    hw = torch.as_tensor(np.asarray(w["head"][0], np.float64))
    hb = torch.as_tensor(np.asarray(w["head"][1], np.float64))
    fwd = [("a1", "e1a", "x"), ("s1", "e1b", "a1"), ("a2", "e2a", "p1"), ("s2", "e2b", "a2"),
           ("a3", "e3a", "p2"), ("s3", "e3b", "a3"), ("a4", "e4a", "p3"), ("b4", "e4b", "a4"),
           ("a5", "d3a", "c3"), ("b5", "d3b", "a5"), ("a6", "d2a", "c2"), ("b6", "d2b", "a6"),
           ("a7", "d1a", "c1"), ("b7", "d1b", "a7")]
    for out, name, inp in fwd:
        _stored_close(A[out], unet.conv_layer(A[inp], *W[name]), f"forward {name}")
    for out, inp in (("p1", "s1"), ("p2", "s2"), ("p3", "s3")):
        _stored_close(A[out], unet.pool_layer(A[inp]), f"pool {out}")
    for cat, up, skip in (("c3", "b4", "s3"), ("c2", "b5", "s2"), ("c1", "b6", "s1")):
        assert torch.equal(A[cat], torch.cat([unet.upsample(A[up]), A[skip]], dim=1)), cat
    lg = logits.double().cpu().numpy()
    assert _rel(lg, unet.head_layer(A["b7"], hw, hb).reshape(-1).numpy()) < 1e-6
    t = (lab < 0).astype(np.float64)
    wt = np.where(t > 0, 2.0, 1.0)
    lg64 = lg.astype(np.float64)
    want_loss = np.mean(wt * (np.log1p(np.exp(-np.abs(lg64))) + np.maximum(lg64, 0) - lg64 * t))
    assert abs(float(loss) - want_loss) <= 1e-6 * want_loss

    rec = m.record
    dl, db7 = rec["head"]
    dlt = torch.as_tensor(dl.double().cpu().numpy()).reshape(1, n, n, n)
    ref_db7, hgw, hgb = unet.head_adjoint(dlt, A["b7"], hw)
    _stored_close(T(db7), ref_db7, "head adjoint")
    assert _rel(g["head"][0], hgw.numpy()) < 1e-5 and _rel(g["head"][1], hgb.numpy()) < 1e-5
    bwd = [("d1b", "a7", "b7"), ("d1a", "c1", "a7"), ("d2b", "a6", "b6"), ("d2a", "c2", "a6"),
           ("d3b", "a5", "b5"), ("d3a", "c3", "a5"), ("e4b", "a4", "b4"), ("e4a", "p3", "a4"),
           ("e3b", "a3", "s3"), ("e3a", "p2", "a3"), ("e2b", "a2", "s2"), ("e2a", "p1", "a2"),
           ("e1b", "a1", "s1"), ("e1a", "x", "a1")]
    for name, xin, y in bwd:
        dy, dx = rec[name]
        rdx, gw, gb = unet.conv_adjoint(A[xin], A[y], T(dy), W[name][0], need_dx=dx is not None)
        if dx is not None:
            _stored_close(T(dx), rdx, f"data gradient {name}")
        ew = _rel(g[name][0], unet.from_torch_weight(gw))
        eb = _rel(g[name][1], gb.numpy()) if gb.abs().max() > 0 else 0.0
        log(f"weight gradient {name}: {ew:.2e}, bias {eb:.2e}")
        assert ew < 1e-5 and eb < 1e-5, name
    for key, v in rec.items():
        if isinstance(key, tuple) and key[0] == "up":
            _stored_close(T(v[1]), unet.upsample_adjoint(T(v[0])), f"upsample adjoint {key[1]}")
        elif isinstance(key, tuple) and key[0] == "pool":
            dp, before, after = v
            _stored_close(T(after), unet.pool_adjoint_add(T(dp), T(before)),
                          f"pool adjoint {key[1]}")
    assert sum(isinstance(k, tuple) for k in rec) == 6


def _bf16_grid(shape, seed, lo=-1.0, hi=1.0):
    """Values on a 2^-8 grid in [lo, hi] (exact in BF16, and their sums of
    eight exact in FP32)."""
    v = np.round(np.random.default_rng(seed).uniform(lo, hi, shape) * 256.0) / 256.0
    return v.astype(np.float32)


def test_pool_and_upsample_adjoints_are_their_definitions():
    """Backward of 2x2x2 average pooling: each cell gets 1/8 of its parent's
    gradient; backward of nearest upsampling: each half-size cell gets the
    sum of its 8 children's gradients (both rounded to BF16; exact here)."""
    import torch

    from paper_2208_05524_amd import nn
    L = nn.lib()
    b, d, h, w, c = 2, 6, 4, 10, 24
    dy_small = _bf16_grid((b, d // 2, h // 2, w // 2, c), 11)
    dx = torch.empty((b, d, h, w, c), dtype=torch.bfloat16, device="cuda")
    dys = _dev_bf16(dy_small)
    nn.check(L.vesis_nn_pool2(_stream(), nn.ptr(dys), nn.ptr(dx), b, d, h, w, c, 1), "pool bwd")
    zi, yi, xi = np.meshgrid(np.arange(d) // 2, np.arange(h) // 2, np.arange(w) // 2,
                             indexing="ij")
    want = 0.125 * dy_small[:, zi, yi, xi, :]
    assert np.array_equal(dx.float().cpu().numpy(), want.astype(np.float32))
    dy_full = _bf16_grid((b, d, h, w, c), 12)
    ds = torch.empty((b, d // 2, h // 2, w // 2, c), dtype=torch.bfloat16, device="cuda")
    dyf = _dev_bf16(dy_full)
    nn.check(L.vesis_nn_up2(_stream(), nn.ptr(dyf), nn.ptr(ds), b, d, h, w, c, 1), "up bwd")
    want = dy_full.reshape(b, d // 2, 2, h // 2, 2, w // 2, 2, c).astype(np.float64).sum(
        axis=(2, 4, 6))
    assert np.array_equal(ds.float().cpu().numpy().astype(np.float64), _bf(want))


def test_relu_adjoint_and_head_are_their_definitions():
    """ReLU adjoint: dy where y > 0; head: logit = b + sum_c w_c x_c, its
    input gradient dlogit w_c (rounded to BF16), dw = sum_p dlogit x,
    db = sum_p dlogit."""
    import ctypes

    import torch

    from paper_2208_05524_amd import nn
    L = nn.lib()
    p, c = 3001, 32
    r = np.random.default_rng(13)
    y = _bf(r.standard_normal(p * c))
    dy = _bf(r.standard_normal(p * c))
    g = torch.empty(p * c, dtype=torch.bfloat16, device="cuda")
    yd, dyd = _dev_bf16(y), _dev_bf16(dy)
    nn.check(L.vesis_nn_relu_bwd(_stream(), nn.ptr(yd), nn.ptr(dyd), nn.ptr(g), p * c),
             "relu bwd")
    assert np.array_equal(g.double().cpu().numpy(), np.where(y > 0, dy, 0.0))
    x = _bf(np.abs(r.standard_normal((p, c))))
    hw = r.uniform(-1, 1, c).astype(np.float32)
    hb = np.array([0.3], np.float32)
    xd = _dev_bf16(x)
    wt, bt = torch.tensor(hw, device="cuda"), torch.tensor(hb, device="cuda")
    logits = torch.empty(p, dtype=torch.float32, device="cuda")
    nn.check(L.vesis_nn_head_fwd(_stream(), nn.ptr(xd), nn.ptr(wt), nn.ptr(bt), nn.ptr(logits),
                                 p, c), "head fwd")
    want = hb[0] + x @ hw.astype(np.float64)
    np.testing.assert_allclose(logits.cpu().numpy(), want, rtol=1e-5, atol=1e-6 * np.abs(want).max())
    dl = r.uniform(-1e-3, 1e-3, p).astype(np.float32)
    dlt = torch.tensor(dl, device="cuda")
    dx = torch.empty((p, c), dtype=torch.bfloat16, device="cuda")
    dw = torch.empty(c, dtype=torch.float32, device="cuda")
    db = torch.empty(1, dtype=torch.float32, device="cuda")
    wsb = 4 * c * ((p + 1023) // 1024)
    ws = torch.empty(wsb // 4, dtype=torch.float32, device="cuda")
    nn.check(L.vesis_nn_head_bwd(_stream(), nn.ptr(dlt), nn.ptr(xd), nn.ptr(wt), nn.ptr(dx),
                                 nn.ptr(dw), nn.ptr(db), nn.ptr(ws), ctypes.c_size_t(wsb), p, c),
             "head bwd")
    prod = (dl.astype(np.float64)[:, None] * hw.astype(np.float64)[None, :]).astype(np.float32)
    assert np.array_equal(dx.double().cpu().numpy(), _bf(prod))
    np.testing.assert_allclose(dw.cpu().numpy(), dl.astype(np.float64) @ x, rtol=1e-5,
                               atol=1e-6 * np.abs(dl).sum() * np.abs(x).max())
    assert abs(float(db.item()) - dl.astype(np.float64).sum()) <= 1e-5 * np.abs(dl).sum()


def test_bce_is_its_definition():
    """Mean weighted binary cross-entropy with logits (target 1 where the
    label is -1, weight pos_weight there) and its gradient w (sigmoid(l) - t) / P."""
    import torch

    from paper_2208_05524_amd import nn
    L = nn.lib()
    p = 50001
    r = np.random.default_rng(14)
    lg = r.uniform(-12, 12, p).astype(np.float32)
    lab = np.where(r.random(p) < 0.3, -1, 1).astype(np.int8)
    pw = 2.5
    dl = torch.empty(p, dtype=torch.float32, device="cuda")
    part = torch.empty(333, dtype=torch.float64, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    lgd, labd = torch.tensor(lg, device="cuda"), torch.tensor(lab, device="cuda")
    nn.check(L.vesis_nn_bce(_stream(), nn.ptr(lgd), nn.ptr(labd), p, pw, nn.ptr(dl),
                            nn.ptr(part), 333, nn.ptr(loss)), "bce")
    l64 = lg.astype(np.float64)
    t = (lab < 0).astype(np.float64)
    wt = np.where(t > 0, pw, 1.0)
    want = np.mean(wt * (np.log1p(np.exp(-np.abs(l64))) + np.maximum(l64, 0) - l64 * t))
    assert abs(float(loss.item()) - want) <= 1e-6 * want
    gwant = wt * (1.0 / (1.0 + np.exp(-l64)) - t) / p
    np.testing.assert_allclose(dl.cpu().numpy(), gwant, rtol=1e-5, atol=1e-6 * np.abs(gwant).max())


def test_adam_is_the_published_update():
    """Three Adam steps (Kingma & Ba: m <- b1 m + (1 - b1) g, v <- b2 v +
    (1 - b2) g^2, w <- w - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps))
    against that update in FP64."""
    import torch

    from paper_2208_05524_amd import nn
    L = nn.lib()
    n = 10007
    r = np.random.default_rng(15)
    w = r.standard_normal(n).astype(np.float32)
    # the kernel takes FP32 hyper-parameters: the reference uses those values
    lr, b1, b2, eps = (float(np.float32(v)) for v in (1e-3, 0.9, 0.999, 1e-8))
    wd = torch.tensor(w, device="cuda")
    md = torch.zeros(n, dtype=torch.float32, device="cuda")
    vd = torch.zeros(n, dtype=torch.float32, device="cuda")
    w64, m64, v64 = w.astype(np.float64), np.zeros(n), np.zeros(n)
    mabs = np.zeros(n)   # the same recursion on |g|: the scale of m's rounding
    for step in range(1, 4):
        g = (r.standard_normal(n) * 10.0 ** r.uniform(-4, 0, n)).astype(np.float32)
        gd = torch.tensor(g, device="cuda")
        nn.check(L.vesis_nn_adam(_stream(), nn.ptr(wd), nn.ptr(gd), nn.ptr(md), nn.ptr(vd), n,
                                 lr, b1, b2, eps, step), "adam")
        g64 = g.astype(np.float64)
        m64 = b1 * m64 + (1 - b1) * g64
        mabs = b1 * mabs + (1 - b1) * np.abs(g64)
        v64 = b2 * v64 + (1 - b2) * g64 * g64
        w64 = w64 - lr * (m64 / (1 - b1 ** step)) / (np.sqrt(v64 / (1 - b2 ** step)) + eps)
    # FP32 recursions: a few ulps of the magnitudes they add (m's terms can
    # cancel, v's cannot)
    assert np.all(np.abs(md.cpu().numpy() - m64) <= 1e-6 * mabs)
    np.testing.assert_allclose(vd.cpu().numpy(), v64, rtol=1e-5, atol=0)
    step_sizes = np.abs(w64 - w.astype(np.float64))
    err = np.abs(wd.cpu().numpy().astype(np.float64) - w64)
    # FP32 arithmetic: the weight carries its own rounding (ulp of |w|) plus a
    # small relative error on the step
    assert np.all(err <= 1e-4 * step_sizes + 2.0 * np.spacing(np.abs(w).astype(np.float32)))


def test_trained_network_start_needs_fewer_sweeps():
    """What the network gains: trained on the relaxed labels of 160
    molecules (300 to 1,500 atoms, 64^3 cells of 0.1 nm), its labels start
    the relaxation of 16 held-out molecules closer to equilibrium than the
    tight start: fewer colour sweeps in total, and every relaxation from it
    still ends at a local minimum (zero-flip sweep)."""
    import torch

    from helpers import gpu_context
    from paper_2208_05524_amd.learned import (Sample, UNet, molecule_arrays, predict_logits,
                                              relaxed_labels, train)
    dev = torch.device("cuda")
    train_set = synth.warm_start_set(160, n=64, h=0.1, seed0=5000)
    test_set = synth.warm_start_set(16, n=64, h=0.1, seed0=9000)
    labels, _ = relaxed_labels(train_set)
    samples = [Sample(w, lab, dev) for w, lab in zip(train_set, labels)]
    m = UNet(64, seed=2)
    losses = train(m, samples, steps=4 * len(samples), lr=2e-3)
    log("training loss first/last", np.mean(losses[:20]), np.mean(losses[-20:]))
    tight, learned = [], []
    for w in test_set:
        c = gpu_context(w)
        c.init_labels("tight", 1.0)
        rc, st = c.minimize()
        assert rc == 0
        tight.append(st["sweeps"])
        pos4, sig, q = molecule_arrays(w, dev)
        c.init_labels_logits(predict_logits(m, pos4, sig, q, w.h, w.center))
        rc, st = c.minimize()
        assert rc == 0 and st["converged"] == 1
        learned.append(st["sweeps"])
        c.close()
    log("sweeps to equilibrium, tight start", tight, "learned start", learned)
    log(f"mean {np.mean(tight):.2f} -> {np.mean(learned):.2f}")
    assert sum(learned) < sum(tight)
