"""The allocation-free forward pass of the initial-guess network
(iim_net_forward_noalloc, called through the C ABI) against the allocating
one (iim_net_forward) on the same network and inputs: the same kernels, so
the outputs must be identical.  Two calls in a row, the second with a
smaller input (the shared scratch keeps the first call's contents), in BF16
and FP32 operands; sizes beyond the scratch limit are refused."""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_2109_13628_amd as iim

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _segments(lengths):
    seg0, segl, pos, start = [], [], [], 0
    for L in lengths:
        for q in range(L):
            seg0.append(start)
            segl.append(L)
            pos.append(q)
        start += L
    return torch.as_tensor(np.array([seg0, segl, pos], dtype=np.int32), device=DEV)


def _forward(fn, net, x, seq, B, P):
    y = torch.full((B, P), float("nan"), dtype=torch.float32, device=DEV)
    rc = fn(net._h, C.c_void_p(x.data_ptr()), B, P, C.c_void_p(seq.data_ptr()), C.c_void_p(y.data_ptr()))
    assert rc == iim.IIM_OK, (rc, iim.lib().iim_last_error(None))
    torch.cuda.synchronize()
    return y


@pytest.mark.parametrize("bf16", [True, False])
def test_noalloc_forward_matches_allocating_forward(bf16):
    L = iim.lib()
    net = iim.Network(width=128, layers=4, bf16=bf16, seed=3)
    gen = torch.Generator(device="cpu").manual_seed(11)
    # the second call is smaller than the first
    for lengths, B in (([37, 50, 3, 1, 70, 200], 9), ([64, 5], 2)):
        P = sum(lengths)
        seq = _segments(lengths)
        x = torch.randn((B, P, iim.NET_FEATURES), generator=gen).to(DEV)
        y_ref = _forward(L.iim_net_forward, net, x, seq, B, P)
        y = _forward(L.iim_net_forward_noalloc, net, x, seq, B, P)
        assert torch.isfinite(y_ref).all()
        assert torch.equal(y, y_ref), float((y - y_ref).abs().max())
    net.close()


def test_noalloc_forward_refuses_sizes_beyond_the_limit():
    L = iim.lib()
    net = iim.Network(width=128, layers=4, bf16=True, seed=1)
    limit = (4 << 20) // (2 * 128)
    P = 1024
    B = limit // P + 1
    seq = _segments([P])
    one = C.c_void_p(1)
    rc = L.iim_net_forward_noalloc(net._h, one, B, P, C.c_void_p(seq.data_ptr()), one)
    assert rc == iim.IIM_EINVAL
    net.close()
