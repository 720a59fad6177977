"""The allocation-free head gradient (vesis_nn_head_bwd_noalloc), called
through the C ABI, against the workspace entry point vesis_nn_head_bwd on
the same inputs: identical results, on two calls in a row (the second with
fewer positions and channels, so it reads the static scratch the first call
left), and the size limit refused before anything is launched."""
import ctypes as C

import numpy as np
import pytest

import synth
from helpers import log

pytestmark = pytest.mark.gpu


def _inputs(p, c, seed):
    import torch
    rng = synth.SplitMix64(seed)
    dlogit = torch.from_numpy(rng.uniform(p, -1e-3, 1e-3).astype(np.float32)).cuda()
    x = torch.from_numpy(rng.uniform(p * c, -2.0, 2.0).astype(np.float32)).cuda()
    x = x.to(torch.bfloat16).reshape(p, c).contiguous()
    w = torch.from_numpy(rng.uniform(c, -0.5, 0.5).astype(np.float32)).cuda()
    return dlogit, x, w


def _outputs(p, c):
    import torch
    dx = torch.full((p, c), float("nan"), dtype=torch.bfloat16, device="cuda")
    dw = torch.full((c,), float("nan"), dtype=torch.float32, device="cuda")
    db = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
    return dx, dw, db


def test_head_bwd_noalloc_equals_workspace_entry_point():
    import torch

    from paper_2208_05524_amd import nn
    L = nn.lib()
    for call, (p, c, seed) in enumerate([(70001, 32, 7001), (5003, 16, 7002)]):
        log(f"no-alloc head gradient call {call}: p={p} c={c}")
        dlogit, x, w = _inputs(p, c, seed)
        st = nn.stream_of(x)
        ref = _outputs(p, c)
        wsb = 4 * c * ((p + 1023) // 1024)
        ws = torch.empty(wsb // 4, dtype=torch.float32, device="cuda")
        nn.check(L.vesis_nn_head_bwd(st, nn.ptr(dlogit), nn.ptr(x), nn.ptr(w), nn.ptr(ref[0]),
                                     nn.ptr(ref[1]), nn.ptr(ref[2]), nn.ptr(ws), wsb, p, c),
                 "head_bwd")
        got = _outputs(p, c)
        nn.check(L.vesis_nn_head_bwd_noalloc(st, nn.ptr(dlogit), nn.ptr(x), nn.ptr(w),
                                             nn.ptr(got[0]), nn.ptr(got[1]), nn.ptr(got[2]), p, c),
                 "head_bwd_noalloc")
        torch.cuda.synchronize()
        for r, g in zip(ref, got):
            assert torch.equal(r, g)
        # and what the gradient is: dw = sum_p dlogit x, db = sum_p dlogit
        xd = x.double().cpu().numpy()
        dl = dlogit.double().cpu().numpy()
        np.testing.assert_allclose(got[1].double().cpu().numpy(), dl @ xd, rtol=1e-4,
                                   atol=1e-6 * np.abs(dl).sum() * np.abs(xd).max())
        assert abs(float(got[2].item()) - dl.sum()) <= 1e-5 * np.abs(dl).sum()


def test_head_bwd_noalloc_refuses_inputs_beyond_its_scratch():
    from paper_2208_05524_amd import nn
    L = nn.lib()
    dlogit, x, w = _inputs(64, 32, 7003)
    dx, dw, db = _outputs(64, 32)
    p_big = 1024 * (262144 // 32) + 1     # one chunk more than the scratch holds at c = 32
    rc = L.vesis_nn_head_bwd_noalloc(nn.stream_of(x), nn.ptr(dlogit), nn.ptr(x), nn.ptr(w),
                                     nn.ptr(dx), nn.ptr(dw), nn.ptr(db), p_big, 32)
    assert rc == -7
    assert bool(dw.isnan().all())        # nothing was launched
