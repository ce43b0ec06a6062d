"""pat_conv3d_forward_static (no workspace, no allocation) against pat_conv3d_forward.

Both entry points are called through the C ABI on the same inputs; they run the
same kernels, so the outputs must be equal bit for bit. Two calls in a row, the
second with a smaller layer (fewer channels, a smaller grid and batch), check
that the per-GPU array is reused correctly; a layer whose packed weights exceed
the array is rejected before anything is enqueued; a layer with more than 64
input channels (unpacked path, no scratch) works too.
"""

import ctypes as C

import pytest
import torch

pytestmark = pytest.mark.gpu


def _both(nb, ci, co, shape, relu, seed):
    from paper_1605_00133_amd import nn
    from paper_1605_00133_amd import pat as P
    g = torch.Generator().manual_seed(seed)
    dev = torch.device("cuda:0")
    x = torch.randn((nb, ci) + shape, generator=g).to(dev)
    w = (0.2 * torch.randn((co, ci, 3, 3, 3), generator=g)).to(dev)
    b = torch.randn(co, generator=g).to(dev)
    y_ref = nn.conv3d_forward(x, w, b, relu=relu)
    y = torch.full_like(y_ref, float("nan"))
    st = torch.cuda.current_stream(dev).cuda_stream
    status = nn.lib().pat_conv3d_forward_static(C.c_void_p(x.data_ptr()), C.c_void_p(w.data_ptr()),
                                                C.c_void_p(b.data_ptr()), C.c_void_p(y.data_ptr()), nb, ci, co,
                                                *shape, 1 if relu else 0, C.c_void_p(st))
    assert status == 0, P.lib().pat_last_error()
    torch.cuda.synchronize()
    return y, y_ref


def test_static_forward_equals_workspace_forward_twice():
    y1, r1 = _both(2, 24, 40, (9, 20, 37), True, 1)          # 3 channel tiles, ragged x and y tiles
    y2, r2 = _both(1, 5, 7, (4, 6, 17), False, 2)            # smaller: fewer tiles, padded channels
    print(f"static vs workspace: max |diff| {float((y1 - r1).abs().max())}, {float((y2 - r2).abs().max())}")
    assert torch.equal(y1, r1) and torch.equal(y2, r2)


def test_static_forward_wide_input_and_limits():
    from paper_1605_00133_amd import nn
    from paper_1605_00133_amd import pat as P
    y, r = _both(1, 72, 16, (3, 5, 18), True, 3)               # > 64 input channels: unpacked, no scratch
    assert torch.equal(y, r)
    lib = nn.lib()
    dev = torch.device("cuda:0")
    x = torch.zeros((1, 64, 2, 2, 2), device=dev)
    w = torch.zeros((512, 64, 3, 3, 3), device=dev)
    out = torch.zeros((1, 512, 2, 2, 2), device=dev)
    st = lib.pat_conv3d_forward_static(C.c_void_p(x.data_ptr()), C.c_void_p(w.data_ptr()), None,
                                       C.c_void_p(out.data_ptr()), 1, 64, 512, 2, 2, 2, 0, None)
    assert st == 1 and b"static scratch holds" in P.lib().pat_last_error()
    assert lib.pat_conv3d_forward_static(None, None, None, None, 0, 4, 4, 2, 2, 2, 0, None) == 0   # empty batch
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0
