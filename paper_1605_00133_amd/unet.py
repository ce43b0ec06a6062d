"""3-level 3D U-Net of the learned update step (not part of the paper's method),
forward and hand-written backward on libpat's kernels.

With widths (c1, c2, c3) = (16, 32, 64) and x = [p_k, z_k] (2 channels):
    level 1 (N):   A1 = relu(conv(x, 2->c1)),          A2 = relu(conv(A1, c1->c1))
    level 2 (N/2): A3 = relu(conv(pool(A2), c1->c2)),  A4 = relu(conv(A3, c2->c2))
    level 3 (N/4): A5 = relu(conv(pool(A4), c2->c3)),  A6 = relu(conv(A5, c3->c3))
    up to N/2:     A7 = relu(conv(up(A6), c3->c2) + A4), A8 = relu(conv(A7, c2->c2))
    up to N:       A9 = relu(conv(up(A8), c2->c1) + A2), A10 = relu(conv(A9, c1->c1))
    output:        O = conv(A10, c1->1)
conv is 3x3x3 with one voxel of zero padding and a bias (BF16 operands on the
matrix cores, FP32 sums), pool the 2x2x2 mean, up nearest-neighbour x2; the skip
connections are added. 319 569 parameters at (16, 32, 64).

backward() runs the chain rule layer by layer from the activations kept by
forward(keep=True): the ReLU masks come from the layers' outputs, the convolution
input and weight gradients from pat_conv3d_backward_*, the resampling adjoints
from pat_pool2_backward / pat_upsample2_backward, and the two skip gradients
are added where the pooled path returns. Every operation is a libpat kernel.
"""

import math

import torch

from . import nn

LAYERS = ("c1", "c2", "c3", "c4", "c5", "c6", "c7", "c8", "c9", "c10", "c11")


def layer_channels(widths=(16, 32, 64)):
    a, b, c = widths
    return {"c1": (2, a), "c2": (a, a), "c3": (a, b), "c4": (b, b), "c5": (b, c), "c6": (c, c),
            "c7": (c, b), "c8": (b, b), "c9": (b, a), "c10": (a, a), "c11": (a, 1)}


class UNet:
    """Weights (device tensors) and the forward / backward passes."""

    def __init__(self, widths=(16, 32, 64), seed=0, device="cuda:0", out_gain=0.1):
        self.widths = tuple(int(w) for w in widths)
        g = torch.Generator().manual_seed(seed)
        self.params = {}
        for name, (ci, co) in layer_channels(self.widths).items():
            gain = out_gain if name == "c11" else 1.0
            w = torch.randn((co, ci, 3, 3, 3), generator=g) * (gain * math.sqrt(2.0 / (ci * 27)))
            self.params[name] = [w.float().to(device).contiguous(), torch.zeros(co, device=device)]
        self._cache = None

    @property
    def n_params(self):
        return sum(w.numel() + b.numel() for w, b in self.params.values())

    def state_dict(self):
        return {f"{k}.{i}": t.detach().cpu() for k, wb in self.params.items() for i, t in enumerate(wb)}

    def load_state_dict(self, sd):
        for k, wb in self.params.items():
            for i in range(2):
                src = sd[f"{k}.{i}"]
                if tuple(src.shape) != tuple(wb[i].shape):
                    raise ValueError(f"{k}.{i}: shape {tuple(src.shape)}, expected {tuple(wb[i].shape)}")
                wb[i].copy_(src.to(wb[i].device, torch.float32))

    def _conv(self, x, name, relu):
        w, b = self.params[name]
        return nn.conv3d_forward(x, w, b, relu=relu)

    def forward(self, x, keep=False):
        """O = net(x) for x [B, 2, N, N, N] (N divisible by 4); keeps the activations for backward()."""
        if x.dim() != 5 or x.shape[1] != 2 or any(int(s) % 4 for s in x.shape[2:]):
            raise ValueError("x must be [B, 2, nz, ny, nx] with sizes divisible by 4")
        a1 = self._conv(x, "c1", True)
        a2 = self._conv(a1, "c2", True)
        p1 = nn.pool2(a2)
        a3 = self._conv(p1, "c3", True)
        a4 = self._conv(a3, "c4", True)
        p2 = nn.pool2(a4)
        a5 = self._conv(p2, "c5", True)
        a6 = self._conv(a5, "c6", True)
        u2 = nn.upsample2(a6)
        a7 = nn.add_act(self._conv(u2, "c7", False), a4, relu=True)
        a8 = self._conv(a7, "c8", True)
        u1 = nn.upsample2(a8)
        a9 = nn.add_act(self._conv(u1, "c9", False), a2, relu=True)
        a10 = self._conv(a9, "c10", True)
        out = self._conv(a10, "c11", False)
        self._cache = dict(x=x, a1=a1, a2=a2, p1=p1, a3=a3, a4=a4, p2=p2, a5=a5, a6=a6, u2=u2, a7=a7, a8=a8, u1=u1,
                           a9=a9, a10=a10) if keep else None
        return out

    def backward(self, d_out):
        """Gradients {name: (dw, db)} of sum(d_out * O) for the last forward(keep=True)."""
        c = self._cache
        if c is None:
            raise RuntimeError("backward() needs forward(keep=True) first")
        W = {k: wb[0] for k, wb in self.params.items()}
        grads = {}

        def layer(name, inp, g):   # weight gradient of a layer, then its input gradient
            grads[name] = nn.conv3d_backward_weight(inp, g, W[name].shape[0])
            return nn.conv3d_backward_input(g, W[name])

        g = layer("c11", c["a10"], d_out.contiguous())
        nn.relu_backward_(c["a10"], g)
        g = layer("c10", c["a9"], g)
        nn.relu_backward_(c["a9"], g)             # gradient of conv9's output and of the skip from A2
        skip2 = g
        g = nn.upsample2_backward(layer("c9", c["u1"], g))
        nn.relu_backward_(c["a8"], g)
        g = layer("c8", c["a7"], g)
        nn.relu_backward_(c["a7"], g)             # gradient of conv7's output and of the skip from A4
        skip4 = g
        g = nn.upsample2_backward(layer("c7", c["u2"], g))
        nn.relu_backward_(c["a6"], g)
        g = layer("c6", c["a5"], g)
        nn.relu_backward_(c["a5"], g)
        g = nn.pool2_backward(layer("c5", c["p2"], g))
        nn.add_act(g, skip4, out=g)
        nn.relu_backward_(c["a4"], g)
        g = layer("c4", c["a3"], g)
        nn.relu_backward_(c["a3"], g)
        g = nn.pool2_backward(layer("c3", c["p1"], g))
        nn.add_act(g, skip2, out=g)
        nn.relu_backward_(c["a2"], g)
        g = layer("c2", c["a1"], g)
        nn.relu_backward_(c["a1"], g)
        grads["c1"] = nn.conv3d_backward_weight(c["x"], g, W["c1"].shape[0])
        return grads
