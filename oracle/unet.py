"""The learned update network (a 3-level 3D U-Net) and its loss, in FP64 with
plain PyTorch CPU operations; gradients by torch's automatic differentiation.

Oracle module: test infrastructure only, never called by the GPU path.

Not part of the paper's method: a network that maps the iterate p_k and the
gradient step z_k = p_k - eta A^T C^T (C A p_k - f) (eq. BP) to
p_{k+1} = max(0, z_k + net([p_k, z_k])). With widths (c1, c2, c3):
    level 1 (N):   A1 = relu(conv(x, 2->c1)), A2 = relu(conv(A1, c1->c1))
    level 2 (N/2): A3 = relu(conv(pool(A2), c1->c2)), A4 = relu(conv(A3, c2->c2))
    level 3 (N/4): A5 = relu(conv(pool(A4), c2->c3)), A6 = relu(conv(A5, c3->c3))
    up to N/2:     A7 = relu(conv(up(A6), c3->c2) + A4), A8 = relu(conv(A7, c2->c2))
    up to N:       A9 = relu(conv(up(A8), c2->c1) + A2), A10 = relu(conv(A9, c1->c1))
    output:        O = conv(A10, c1->1)
conv: 3x3x3 cross-correlation with one voxel of zero padding plus a bias; pool:
2x2x2 mean; up: nearest-neighbour x2; the skip connections are added, not
concatenated. Loss: mean((p_{k+1} - target)^2) over all voxels.
"""

import numpy as np

LAYERS = ("c1", "c2", "c3", "c4", "c5", "c6", "c7", "c8", "c9", "c10", "c11")


def layer_channels(widths=(16, 32, 64)):
    a, b, c = widths
    return {"c1": (2, a), "c2": (a, a), "c3": (a, b), "c4": (b, b), "c5": (b, c), "c6": (c, c),
            "c7": (c, b), "c8": (b, b), "c9": (b, a), "c10": (a, a), "c11": (a, 1)}


def n_params(widths=(16, 32, 64)):
    return sum(ci * co * 27 + co for ci, co in layer_channels(widths).values())


def _torch():
    import torch
    return torch


def net(params, x):
    """O = net(x) for x [B][2][N][N][N]; params: name -> (w [co][ci][3][3][3], b [co]) torch FP64 tensors."""
    torch = _torch()
    F = torch.nn.functional

    def conv(t, name):
        w, b = params[name]
        return F.conv3d(t, w, b, padding=1)

    def pool(t):
        return F.avg_pool3d(t, 2)

    def up(t):
        return F.interpolate(t, scale_factor=2, mode="nearest")

    a1 = torch.relu(conv(x, "c1"))
    a2 = torch.relu(conv(a1, "c2"))
    a3 = torch.relu(conv(pool(a2), "c3"))
    a4 = torch.relu(conv(a3, "c4"))
    a5 = torch.relu(conv(pool(a4), "c5"))
    a6 = torch.relu(conv(a5, "c6"))
    a7 = torch.relu(conv(up(a6), "c7") + a4)
    a8 = torch.relu(conv(a7, "c8"))
    a9 = torch.relu(conv(up(a8), "c9") + a2)
    a10 = torch.relu(conv(a9, "c10"))
    return conv(a10, "c11")


def step(params, p, z):
    """p_{k+1} = max(0, z + net([p, z])) for p, z [B][1][N][N][N] (torch FP64)."""
    torch = _torch()
    return torch.clamp_min(z + net(params, torch.cat([p, z], dim=1)), 0.0)


def loss_and_grads(params_np, p, z, target):
    """(loss, p_next, grads) in FP64: params_np name -> (w, b) numpy arrays; p, z, target numpy
    [B][1][N][N][N]; grads name -> (dw, db) numpy arrays of d loss / d params."""
    torch = _torch()
    params = {k: (torch.tensor(w, dtype=torch.float64, requires_grad=True),
                  torch.tensor(b, dtype=torch.float64, requires_grad=True)) for k, (w, b) in params_np.items()}
    tp, tz, tt = (torch.tensor(np.asarray(a), dtype=torch.float64) for a in (p, z, target))
    out = step(params, tp, tz)
    loss = ((out - tt) ** 2).mean()
    loss.backward()
    grads = {k: (w.grad.numpy().copy(), b.grad.numpy().copy()) for k, (w, b) in params.items()}
    return float(loss), out.detach().numpy(), grads
