"""Network layers of a learned update step (not part of the paper's method).

Binding of include/pat_nn.h: 3x3x3 convolutions with BF16 operands on the
matrix cores and FP32 accumulation, their input and weight gradients, the ReLU
backward and an Adam step, all computed by libpat's kernels. This module checks
tensors, passes pointers and the current stream, and wraps the convolution as a
torch autograd function.
"""

import ctypes as C
import threading

import torch

from . import pat as P

_P = C.c_void_p
_I = C.c_int32
SIGNATURES = {
    "pat_conv3d_workspace_bytes": (C.c_size_t, [_I, _I]),
    "pat_conv3d_forward": (C.c_int, [_P, _P, _P, _P, _I, _I, _I, _I, _I, _I, _I, _P, C.c_size_t, _P]),
    "pat_conv3d_forward_static": (C.c_int, [_P, _P, _P, _P, _I, _I, _I, _I, _I, _I, _I, _P]),
    "pat_conv3d_backward_input": (C.c_int, [_P, _P, _P, _I, _I, _I, _I, _I, _I, _P, C.c_size_t, _P]),
    "pat_conv3d_backward_weight_workspace_bytes": (C.c_size_t, [_I, _I, _I, _I, _I, _I]),
    "pat_conv3d_backward_weight": (C.c_int, [_P, _P, _P, _P, _I, _I, _I, _I, _I, _I, _P, C.c_size_t, _P]),
    "pat_relu_backward": (C.c_int, [_P, _P, C.c_int64, _P]),
    "pat_pool2_forward": (C.c_int, [_P, _P, C.c_int64, _I, _I, _I, _P]),
    "pat_pool2_backward": (C.c_int, [_P, _P, C.c_int64, _I, _I, _I, _P]),
    "pat_upsample2_forward": (C.c_int, [_P, _P, C.c_int64, _I, _I, _I, _P]),
    "pat_upsample2_backward": (C.c_int, [_P, _P, C.c_int64, _I, _I, _I, _P]),
    "pat_add_act": (C.c_int, [_P, _P, _P, C.c_int64, _I, _P]),
    "pat_axpby": (C.c_int, [_P, _P, _P, C.c_int64, C.c_float, C.c_float, _I, _P]),
    "pat_mse_workspace_bytes": (C.c_size_t, []),
    "pat_mse": (C.c_int, [_P, _P, _P, C.c_int64, _I, _P, _P, C.c_size_t, _P]),
    "pat_adam_step": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float, _I, _P]),
}

_bound = False
_bind_lock = threading.Lock()


def lib():
    """libpat.so with the layer signatures bound (once, under a lock, so that
    concurrent first callers never see a half-bound library)."""
    global _bound
    L = P.lib()
    if not _bound:
        with _bind_lock:
            if not _bound:
                for name, (res, args) in SIGNATURES.items():
                    fn = getattr(L, name)
                    fn.restype = res
                    fn.argtypes = args
                _bound = True
    return L


def _ptr(t, name, shape=None, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float32 or t.device.type != "cuda" or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return C.c_void_p(t.data_ptr())


def _stream(t):
    return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _sizes(x, w):
    if x.dim() != 5 or w.dim() != 5 or tuple(w.shape[2:]) != (3, 3, 3):
        raise ValueError("x must be [B, C, nz, ny, nx] and w [c_out, c_in, 3, 3, 3]")
    if x.shape[1] != w.shape[1]:
        raise ValueError(f"x has {x.shape[1]} channels, w expects {w.shape[1]}")
    return (int(x.shape[0]), int(w.shape[1]), int(w.shape[0])) + tuple(int(s) for s in x.shape[2:])


def _workspace(ci, co, device):
    nbytes = lib().pat_conv3d_workspace_bytes(ci, co)
    if nbytes == 0:
        raise ValueError("invalid channel counts")
    return torch.empty(nbytes, dtype=torch.uint8, device=device), nbytes


def conv3d_forward(x, w, bias=None, relu=False):
    """y = conv(x, w) + bias, optionally ReLU; returns a new [B, c_out, nz, ny, nx] tensor."""
    nb, ci, co, nz, ny, nx = _sizes(x, w)
    y = torch.empty((nb, co, nz, ny, nx), dtype=torch.float32, device=x.device)
    bp = None if bias is None else _ptr(bias, "bias", (co,), x.device)
    ws, nbytes = _workspace(ci, co, x.device)
    P._check(lib().pat_conv3d_forward(_ptr(x, "x"), _ptr(w, "w", device=x.device), bp, _ptr(y, "y"), nb, ci, co,
                                      nz, ny, nx, 1 if relu else 0, C.c_void_p(ws.data_ptr()), nbytes, _stream(x)))
    return y


def conv3d_forward_static(x, w, bias=None, relu=False, out=None):
    """As conv3d_forward through pat_conv3d_forward_static: no workspace, the packed
    weights go to the library's own per-GPU array. Writes `out` when given (so a
    caller under graph capture allocates nothing here) and returns it."""
    nb, ci, co, nz, ny, nx = _sizes(x, w)
    y = torch.empty((nb, co, nz, ny, nx), dtype=torch.float32, device=x.device) if out is None else out
    bp = None if bias is None else _ptr(bias, "bias", (co,), x.device)
    P._check(lib().pat_conv3d_forward_static(_ptr(x, "x"), _ptr(w, "w", device=x.device), bp,
                                             _ptr(y, "y", (nb, co, nz, ny, nx), x.device), nb, ci, co, nz, ny, nx,
                                             1 if relu else 0, _stream(x)))
    return y


def conv3d_backward_input(dy, w):
    """dx = the adjoint of x -> conv(x, w) applied to dy."""
    nb, co = int(dy.shape[0]), int(w.shape[0])
    if dy.dim() != 5 or dy.shape[1] != co:
        raise ValueError("dy must be [B, c_out, nz, ny, nx]")
    ci = int(w.shape[1])
    nz, ny, nx = (int(s) for s in dy.shape[2:])
    dx = torch.empty((nb, ci, nz, ny, nx), dtype=torch.float32, device=dy.device)
    ws, nbytes = _workspace(ci, co, dy.device)
    P._check(lib().pat_conv3d_backward_input(_ptr(dy, "dy"), _ptr(w, "w", device=dy.device), _ptr(dx, "dx"), nb, ci,
                                             co, nz, ny, nx, C.c_void_p(ws.data_ptr()), nbytes, _stream(dy)))
    return dx


def conv3d_backward_weight(x, dy, c_out=None):
    """(dw, dbias): gradients of sum(dy * conv(x, w)) with respect to w and the bias."""
    nb, ci = int(x.shape[0]), int(x.shape[1])
    co = int(dy.shape[1]) if c_out is None else int(c_out)
    nz, ny, nx = (int(s) for s in x.shape[2:])
    _ptr(dy, "dy", (nb, co, nz, ny, nx), x.device)
    nbytes = lib().pat_conv3d_backward_weight_workspace_bytes(nb, ci, co, nz, ny, nx)
    if nbytes == 0:
        raise ValueError("invalid convolution sizes")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    dw = torch.empty((co, ci, 3, 3, 3), dtype=torch.float32, device=x.device)
    db = torch.empty((co,), dtype=torch.float32, device=x.device)
    P._check(lib().pat_conv3d_backward_weight(_ptr(x, "x"), _ptr(dy, "dy"), _ptr(dw, "dw"), _ptr(db, "db"), nb, ci,
                                              co, nz, ny, nx, C.c_void_p(ws.data_ptr()), nbytes, _stream(x)))
    return dw, db


def relu_backward_(y, g):
    """g[y <= 0] = 0 in place."""
    if y.shape != g.shape:
        raise ValueError("y and g must have the same shape")
    P._check(lib().pat_relu_backward(_ptr(y, "y"), _ptr(g, "g", device=y.device), y.numel(), _stream(y)))
    return g


def adam_step_(w, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place on w, m, v (step counts from 1)."""
    for t, n in ((g, "g"), (m, "m"), (v, "v")):
        _ptr(t, n, w.shape, w.device)
    P._check(lib().pat_adam_step(_ptr(w, "w"), _ptr(g, "g"), _ptr(m, "m"), _ptr(v, "v"), w.numel(), float(lr),
                                 float(beta1), float(beta2), float(eps), int(step), _stream(w)))


def _vol(t, name):
    if t.dim() != 5:
        raise ValueError(f"{name} must be [B, C, nz, ny, nx]")
    return int(t.shape[0]) * int(t.shape[1]), tuple(int(s) for s in t.shape[2:])


def pool2(x):
    """2x2x2 average pooling: [B, C, nz, ny, nx] (even sizes) -> [B, C, nz/2, ny/2, nx/2]."""
    ch, (nz, ny, nx) = _vol(x, "x")
    y = torch.empty(x.shape[:2] + (nz // 2, ny // 2, nx // 2), dtype=torch.float32, device=x.device)
    P._check(lib().pat_pool2_forward(_ptr(x, "x"), _ptr(y, "y"), ch, nz, ny, nx, _stream(x)))
    return y


def pool2_backward(dy):
    """Adjoint of pool2: [B, C, n/2 ...] -> [B, C, n ...], each child dy(parent) / 8."""
    ch, (nz, ny, nx) = _vol(dy, "dy")
    dx = torch.empty(dy.shape[:2] + (2 * nz, 2 * ny, 2 * nx), dtype=torch.float32, device=dy.device)
    P._check(lib().pat_pool2_backward(_ptr(dy, "dy"), _ptr(dx, "dx"), ch, 2 * nz, 2 * ny, 2 * nx, _stream(dy)))
    return dx


def upsample2(x):
    """Nearest-neighbour x2 upsampling: [B, C, nz, ny, nx] -> [B, C, 2nz, 2ny, 2nx]."""
    ch, (nz, ny, nx) = _vol(x, "x")
    y = torch.empty(x.shape[:2] + (2 * nz, 2 * ny, 2 * nx), dtype=torch.float32, device=x.device)
    P._check(lib().pat_upsample2_forward(_ptr(x, "x"), _ptr(y, "y"), ch, nz, ny, nx, _stream(x)))
    return y


def upsample2_backward(dy):
    """Adjoint of upsample2: the sum over the 8 children, [B, C, 2n ...] -> [B, C, n ...]."""
    ch, (nz, ny, nx) = _vol(dy, "dy")
    dx = torch.empty(dy.shape[:2] + (nz // 2, ny // 2, nx // 2), dtype=torch.float32, device=dy.device)
    P._check(lib().pat_upsample2_backward(_ptr(dy, "dy"), _ptr(dx, "dx"), ch, nz // 2, ny // 2, nx // 2,
                                          _stream(dy)))
    return dx


def add_act(a, b=None, relu=False, out=None):
    """act(a + b) (b may be None); out may be a or b (in place)."""
    y = torch.empty_like(a) if out is None else out
    bp = None if b is None else _ptr(b, "b", a.shape, a.device)
    P._check(lib().pat_add_act(_ptr(a, "a"), bp, _ptr(y, "y", a.shape, a.device), a.numel(), 1 if relu else 0,
                               _stream(a)))
    return y


def axpby(x, y=None, alpha=1.0, beta=1.0, clamp0=False, out=None):
    """alpha x + beta y (y may be None), optionally max(., 0); out may be x or y (in place)."""
    o = torch.empty_like(x) if out is None else out
    yp = None if y is None else _ptr(y, "y", x.shape, x.device)
    P._check(lib().pat_axpby(_ptr(x, "x"), yp, _ptr(o, "out", x.shape, x.device), x.numel(), float(alpha),
                             float(beta), 1 if clamp0 else 0, _stream(x)))
    return o


def mse(a, t, grad=None, mask0=False):
    """Mean squared error of a against t as a device FP64 scalar tensor; fills `grad` (if given)
    with 2 (a - t) / n, zero where a <= 0 when mask0."""
    loss = torch.empty((), dtype=torch.float64, device=a.device)
    nbytes = lib().pat_mse_workspace_bytes()
    ws = torch.empty(nbytes, dtype=torch.uint8, device=a.device)
    gp = None if grad is None else _ptr(grad, "grad", a.shape, a.device)
    P._check(lib().pat_mse(_ptr(a, "a"), _ptr(t, "t", a.shape, a.device), gp, a.numel(), 1 if mask0 else 0,
                           C.c_void_p(loss.data_ptr()), C.c_void_p(ws.data_ptr()), nbytes, _stream(a)))
    return loss


class _Conv3d(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, w, bias, relu):
        x, w = x.detach().contiguous(), w.detach().contiguous()
        y = conv3d_forward(x, w, None if bias is None else bias.detach().contiguous(), relu)
        ctx.relu, ctx.has_bias = relu, bias is not None
        ctx.save_for_backward(x, w, y)
        return y

    @staticmethod
    def backward(ctx, gy):
        x, w, y = ctx.saved_tensors
        g = gy.contiguous().clone() if ctx.relu else gy.contiguous()
        if ctx.relu:
            relu_backward_(y, g)
        dx = conv3d_backward_input(g, w) if ctx.needs_input_grad[0] else None
        dw, db = conv3d_backward_weight(x, g, w.shape[0]) if (ctx.needs_input_grad[1] or ctx.needs_input_grad[2]) \
            else (None, None)
        return dx, dw, db if ctx.has_bias else None, None


def conv3d(x, w, bias=None, relu=False):
    """Differentiable BF16-MFMA convolution (3x3x3, zero padding 1) with optional ReLU."""
    return _Conv3d.apply(x, w, bias, relu)


def bench_layers(shapes=((8, 2, 24, 32), (8, 24, 24, 32), (8, 24, 1, 32), (1, 16, 16, 128)), reps=20):
    """HIP-event timings (us per call) of forward, input gradient and weight gradient
    for [batch, c_in, c_out, n^3] layers on random data; one host thread, one stream."""
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev).manual_seed(0)
    out = []

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3

    for nb, ci, co, n in shapes:
        x = torch.randn((nb, ci, n, n, n), generator=g, device=dev)
        w = torch.randn((co, ci, 3, 3, 3), generator=g, device=dev)
        b = torch.randn((co,), generator=g, device=dev)
        dy = torch.randn((nb, co, n, n, n), generator=g, device=dev)
        flop = 2.0 * nb * n ** 3 * ci * co * 27
        r = {"batch": nb, "c_in": ci, "c_out": co, "n": n,
             "forward_us": timed(lambda: conv3d_forward(x, w, b, True)),
             "input_grad_us": timed(lambda: conv3d_backward_input(dy, w)),
             "weight_grad_us": timed(lambda: conv3d_backward_weight(x, dy))}
        r["forward_tflops"] = flop / r["forward_us"] / 1e6
        out.append(r)
    return out


if __name__ == "__main__":
    import json
    for r in bench_layers():
        print(json.dumps({k: (round(v, 2) if isinstance(v, float) else v) for k, v in r.items()}), flush=True)
