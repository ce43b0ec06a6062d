"""3x3x3 convolution layers of a learned update step, in FP64.

Oracle module: test infrastructure only, never called by the GPU path.

Not part of the paper's method. The layer is a cross-correlation with one voxel
of zero padding: y[b][co][z,y,x] = sum over ci, dz, dy, dx in {-1, 0, 1} of
w[co][ci][dz+1][dy+1][dx+1] x[b][ci][z+dz, y+dy, x+dx] (+ bias[co]). The input
gradient is its adjoint, the weight gradient the derivative of sum(dy * y) in w.
bf16 rounds FP32 values to bfloat16 (8 exponent bits, 8 significant bits) to
nearest, ties to even: the precision in which the GPU multiplies.
"""

import numpy as np


def bf16(a):
    """Round to bfloat16 (nearest, ties to even) and return as float64; finite inputs."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _pad(x):
    return np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1), (1, 1)))


def conv3d(x, w, bias=None, relu=False):
    """x [B][ci][nz][ny][nx], w [co][ci][3][3][3] -> [B][co][nz][ny][nx]."""
    x = np.asarray(x, dtype=np.float64)
    nb, ci, nz, ny, nx = x.shape
    xp = _pad(x)
    y = np.zeros((nb, w.shape[0], nz, ny, nx))
    for a in range(3):
        for b in range(3):
            for c in range(3):
                shifted = xp[:, :, a:a + nz, b:b + ny, c:c + nx]
                y += np.einsum("bizyx,oi->bozyx", shifted, w[:, :, a, b, c])
    if bias is not None:
        y += np.asarray(bias, dtype=np.float64)[None, :, None, None, None]
    return np.maximum(y, 0.0) if relu else y


def conv3d_backward_input(dy, w):
    """dx[b][ci][v] = sum_{co, d} w[co][ci][d] dy[b][co][v - d]: scatter each tap back."""
    nb, co, nz, ny, nx = dy.shape
    dxp = np.zeros((nb, w.shape[1], nz + 2, ny + 2, nx + 2))
    for a in range(3):
        for b in range(3):
            for c in range(3):
                dxp[:, :, a:a + nz, b:b + ny, c:c + nx] += np.einsum("bozyx,oi->bizyx", dy, w[:, :, a, b, c])
    return dxp[:, :, 1:-1, 1:-1, 1:-1]


def conv3d_backward_weight(x, dy):
    """(dw, dbias): dw[co][ci][d] = sum_{b,v} dy[b][co][v] x[b][ci][v + d], dbias[co] = sum dy[b][co][v]."""
    nb, ci, nz, ny, nx = x.shape
    xp = _pad(np.asarray(x, dtype=np.float64))
    dw = np.zeros((dy.shape[1], ci, 3, 3, 3))
    for a in range(3):
        for b in range(3):
            for c in range(3):
                dw[:, :, a, b, c] = np.einsum("bozyx,bizyx->oi", dy, xp[:, :, a:a + nz, b:b + ny, c:c + nx])
    return dw, dy.sum(axis=(0, 2, 3, 4))


def adam_step(w, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma and Ba): returns the new (w, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v


def pool2(x):
    """2x2x2 average pooling over the last three axes (even sizes): the mean of the 8 children."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros(x.shape[:-3] + tuple(s // 2 for s in x.shape[-3:]))
    for a in range(2):
        for b in range(2):
            for c in range(2):
                out += x[..., a::2, b::2, c::2]
    return out / 8.0


def upsample2(x):
    """Nearest-neighbour x2 upsampling over the last three axes: every child takes its parent's value."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros(x.shape[:-3] + tuple(2 * s for s in x.shape[-3:]))
    for a in range(2):
        for b in range(2):
            for c in range(2):
                out[..., a::2, b::2, c::2] = x
    return out


def pool2_backward(dy):
    """Adjoint of pool2: each child receives its parent's value / 8."""
    return upsample2(dy) / 8.0


def upsample2_backward(dy):
    """Adjoint of upsample2: the sum over the 8 children."""
    return 8.0 * pool2(dy)
