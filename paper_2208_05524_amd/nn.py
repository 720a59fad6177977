"""ctypes binding of include/vesis_nn.h (layers of the learned warm start).

Argument marshalling only: tensors are torch CUDA tensors used as device
memory; every layer runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C

from . import _lib

NN_EXPORTS = ["vesis_nn_conv3_fwd", "vesis_nn_conv3_fwd_upcat", "vesis_nn_wgrad_workspace", "vesis_nn_conv3_wgrad",
              "vesis_nn_prep_weights", "vesis_nn_relu_bwd", "vesis_nn_pool2", "vesis_nn_up2",
              "vesis_nn_concat", "vesis_nn_split", "vesis_nn_add", "vesis_nn_head_fwd",
              "vesis_nn_head_bwd", "vesis_nn_head_bwd_noalloc",
              "vesis_nn_bce", "vesis_nn_adam", "vesis_nn_featurize"]

_NN = None


class NNError(RuntimeError):
    pass


def lib():
    global _NN
    if _NN is None:
        L = _lib.load()
        P, I, I64, F, D = C.c_void_p, C.c_int, C.c_int64, C.c_float, C.c_double
        L.vesis_nn_conv3_fwd.argtypes = [P, P, P, P, P, I, I, I, I, I, I, I]
        L.vesis_nn_conv3_fwd_upcat.argtypes = [P, P, I, P, I, P, P, P, I, I, I, I, I, I]
        L.vesis_nn_wgrad_workspace.argtypes = [I, I, I, I, I, I, C.POINTER(C.c_size_t)]
        L.vesis_nn_conv3_wgrad.argtypes = [P, P, P, P, P, P, C.c_size_t, I, I, I, I, I, I]
        L.vesis_nn_prep_weights.argtypes = [P, P, I, I, P, P]
        L.vesis_nn_relu_bwd.argtypes = [P, P, P, P, I64]
        L.vesis_nn_pool2.argtypes = [P, P, P, I, I, I, I, I, I]
        L.vesis_nn_up2.argtypes = [P, P, P, I, I, I, I, I, I]
        L.vesis_nn_concat.argtypes = [P, P, I, P, I, P, I64]
        L.vesis_nn_split.argtypes = [P, P, I, I, P, P, I, I64]
        L.vesis_nn_add.argtypes = [P, P, P, P, I64]
        L.vesis_nn_head_fwd.argtypes = [P, P, P, P, P, I64, I]
        L.vesis_nn_head_bwd.argtypes = [P, P, P, P, P, P, P, P, C.c_size_t, I64, I]
        L.vesis_nn_head_bwd_noalloc.argtypes = [P, P, P, P, P, P, P, I64, I]
        L.vesis_nn_bce.argtypes = [P, P, P, I64, F, P, P, I, P]
        L.vesis_nn_adam.argtypes = [P, P, P, P, P, I64, F, F, F, F, I]
        L.vesis_nn_featurize.argtypes = [P, P, P, P, I64, I, D, P, I, P]
        for n in NN_EXPORTS:
            getattr(L, n).restype = C.c_int
        _NN = L
    return _NN


def ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def stream_of(t):
    import torch
    return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def check(rc, what):
    if rc != 0:
        raise NNError(f"{what} failed with status {rc}")
